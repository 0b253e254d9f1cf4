// Per-task parameter blocks of the kernels.  A single-task launch passes one by value;
// a grouped launch passes a device array of them plus a GroupMap (group.h).
#pragma once
#include <stdint.h>
#include "gemm_f32.h"
#include "group.h"

namespace kfac {

struct EaOut {
  float* F; long ldf; uint16_t* Fb; long ldfb; int d; float rho, c;
};

// Convolution geometry of an im2col operand: NHWC bf16 input x[B][H][W][C], kernel kh x kw,
// zero padding `pad`, stride `stride`, output Ho x Wo.  Row k of the patch matrix is the
// output position (b, oh, ow) = (k / (Ho Wo), (k / Wo) % Ho, k % Wo); column j is the tap
// and channel (dy, dx, c) = (j / (kw C), (j / C) % kw, j % C), reading
// x[b][oh stride - pad + dy][ow stride - pad + dx][c] (zero outside the image).  C == 0
// marks an ordinary row-major operand.
// Division by an invariant q >= 1 of 0 <= n < 2^31 as a multiply and shift: with
// l = ceil(log2 q) and m = floor(2^(31 + l) / q) + 1, floor(n m / 2^(31 + l)) = floor(n / q)
// (Granlund and Montgomery, division by invariant integers using multiplication, 1994).
struct DivMagic {
  uint64_t m;
  int sh;
};
__host__ __device__ inline DivMagic conv_divisor(int q) {
  int l = 0;
  while ((1LL << l) < q) ++l;
  return DivMagic{(uint64_t)((1ULL << (31 + l)) / (uint64_t)q) + 1, 31 + l};
}
__host__ __device__ inline int conv_div(int n, const DivMagic& d) {
  return (int)(((uint64_t)(uint32_t)n * d.m) >> d.sh);
}

struct ConvGeom {
  int B, H, W, C, kh, kw, pad, stride, Ho, Wo;
  int vec;               // C % 8 == 0 and x 16-byte aligned: 8-channel runs as 16-byte loads
  // n / q for 0 <= n < 2^31 as (n * m) >> sh (conv_divisor), for q = C, kw, Ho Wo, Wo
  DivMagic dC, dKw, dHoWo, dWo;
};

struct EaTask {          // EA update: block (upper tile, K slice)
  GemmP g;
  EaOut o;
  int T;                 // tiles per side
  int nks;               // K slices
  ConvGeom cv;           // C > 0: the activations are the im2col patches of an NHWC input
};

struct OmegaTask {       // Gaussian test matrix: block (row block, column group)
  int d, l, d_pad, l_pad;
  uint32_t k0, k1, stream, inv;
  float* OmT; long ldt; uint16_t* OmTb;
  float* Om; long ldo; uint32_t* words;
};

struct SignTask {        // column sign convention: block (column block, row chunk)
  float* U; long ldu; int d, r;
  float* pval; int* pidx; int nchunks;
};

struct BfGemmTask {      // C = A B^T, bf16 operands, K contiguous: block (flat tile)
  int M, N, K;
  const uint16_t* A; long lda;
  const uint16_t* B; long ldb;
  float* C; long ldc;
  int tiles_m;
};

struct SkinnyTask {      // C[M x N] = A[M x K] B[N x K]^T, M <= 288, bf16: block (N tile, K slice)
  int M, N, K;
  const uint16_t* A; long lda;
  const uint16_t* B; long ldb;
  float* C; long ldc;
  float* part;           // ksplit > 1: [ksplit][M][N] fp32 partial sums
  int ksplit, tiles_n;
};

struct SplitTask {       // C[M x N] = A[M x K] B[N x K]^T, M <= 288, fp32 inputs split into
  int M, N, K;           // bf16 hi + lo pairs: block (N tile, K slice)
  const float* A; long lda;
  const float* B; long ldb;
  float* C; long ldc;
  float* part;           // ksplit > 1: [ksplit][M][N] fp32 partial sums
  int ksplit, tiles_n;
};

struct ReduceTask {      // C = sum over k of part[k] (K-slice partials, in slice order)
  int M, N;
  const float* part;     // [ksplit][M][round_up(N, 4)]
  float* C; long ldc;
  int ksplit;
};

struct LinTask {         // K-FAC linear layer GEMMs on bf16 MFMA: block (flat tile)
  int M, N, K;
  const uint16_t* A; long lda;
  const uint16_t* B; long ldb;
  int b_ones;            // K-major B: implicit ones column at index N - 1
  float* C; long ldc;    // fp32 output (nullable)
  uint16_t* Cb; long ldcb;   // bf16 output (nullable)
  const float* bias;     // per output column (nullable)
  int tiles_m, tiles_n;
  EaOut gam;             // fused backward-factor EA (upper tiles after the plain tiles)
  int gam_T;             // tiles per side of gam (0: none)
  ConvGeom cv;           // C > 0: the K-major B operand is the im2col patches of B (NHWC)
  int nks;               // K slices (1: the epilogue writes C / blends gam directly)
  float* part;           // nks > 1: [tile][slice][128 x 128] raw sums, plain tiles then gam's
};

struct GramP {           // C = A B^T in fp64 from fp32 rows: block (tile, K slice)
  const float* A; long lda;
  const float* B; long ldb;
  int L;                 // rows of A and B (l_pad)
  int K;                 // contraction length (d)
  int sym;               // 1: A == B, only upper tiles
  int ksplit;
  double* part;          // [tile][ks][64*64]
  double* C; long ldc;
  int* status;
};

struct CholInvTask {     // blocked Cholesky + inverse of the l x l Gram (one block)
  double* G; long ldg; int n; long m_rows;   // G: lower triangle overwritten by L
  double* Linv; long ldl; int l_pad;
  double* dsave;                             // n doubles: diagonal of G for the retry
  int* status; int* fail_flag; int attempt;
  // second pass of CholeskyQR2: when the Gram is within tol of I (max entry deviation), set
  // *skip and leave the first pass's basis as it is (null: always factor)
  int* skip; double tol;
};

struct TrmmTask {        // Q^T = L^{-1} Y^T: block (column tile, row tile)
  const double* Li; long ldl; int n;
  const float* Yt; long ldy; int ncols;
  float* Qt; long ldq; uint16_t* Qtb; long ldqb; int l_pad;
  const int* skip;       // set by the Cholesky of this pass: Q^T = Y^T (copy)
};

struct TriMeta {         // tridiagonal eigensolver state (see kernels_eig.hip)
  double* es;            // [n] off-diagonal with negligible entries zeroed
  int* blo;              // [n] first row of the block containing row i
  int* bhi;              // [n] one past the last row of that block
  double* lam;           // [n] eigenvalue of task j
  int* col_task;         // [r] task of output column k (descending order)
  int* cstart;           // [r] 1 if column k starts a new cluster
  double* scal;          // [0] ||T|| bound, [1] pivmin, [2] any-cluster flag
};

struct EigTask {         // one small symmetric eigenproblem
  const double* C; long ldc;      // fp64 input (or null)
  const float* Cf; long ldcf;     // fp32 input (exact regime)
  int n, n_pad, r;
  double* A; double* V; double* diag; double* off;
  double* Z; long ldz;
  TriMeta m;
  double* cl;                     // cluster scratch, 5 n
  float* P; long ldp;             // fp32 eigenvectors (n_pad x r)
  float* D; double* Dd;
  int* status;
  int svd;                        // 1: the input is a Gram W^T W; D gets sqrt(lambda) and
                                  // column k of P is scaled by 1 / sqrt(lambda_k), so that
                                  // W P holds W's leading left singular vectors
};

}  // namespace kfac
