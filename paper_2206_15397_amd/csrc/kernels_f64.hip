// fp64 kernels of the randomized eigendecomposition (Alg. 3):
//  * Gram / projection products  G = A B^T  (A, B: l x d fp32, accumulated in fp64 on
//    v_mfma_f64_16x16x4_f64, split over d with an in-order reduction);
//  * CholeskyQR: blocked right-looking Cholesky of the l x l Gram in one workgroup, with a
//    shifted retry, and the blocked forward substitution Q^T = L^{-1} Y^T;
#include <utility>
#include "kernels.h"

namespace kfac {

// ======================================================================================
// Gram / projection: C[a][b] = sum_k A[a][k] * B[b][k]   (fp32 inputs, fp64 accumulate)
// ======================================================================================
constexpr int GR_T = 64, GR_BK = 16;

__device__ __forceinline__ void tile_of(int t, int T, int sym, int& I, int& J) {
  if (sym) { upper_tile(t, T, I, J); }
  else { I = t / T; J = t % T; }
}

// block (tile, K slice), 256 threads = 2 x 2 waves of 32 x 32.
__device__ __forceinline__ void gram_partial_body(const GramP& p, int bx, int by) {
  __shared__ double sa[GR_BK][GR_T + 2];
  __shared__ double sb[GR_BK][GR_T + 2];
  const int T = (p.L + GR_T - 1) / GR_T;
  int I, J;
  tile_of(bx, T, p.sym, I, J);
  const int a0 = I * GR_T, b0 = J * GR_T;
  const int ks = by, nks = p.ksplit;
  const int kchunk = ((p.K + nks - 1) / nks + GR_BK - 1) / GR_BK * GR_BK;
  const int kb = ks * kchunk, ke = min(p.K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += GR_BK) {
    __syncthreads();
    // 64 rows x 16 k for each operand: 4 elements per thread, consecutive threads -> k
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int e = tid + u * 256;
      int row = e / GR_BK, k = e % GR_BK;
      int gk = k0 + k;
      float va = 0.f, vb = 0.f;
      if (gk < ke) {
        if (a0 + row < p.L) va = p.A[(long)(a0 + row) * p.lda + gk];
        if (b0 + row < p.L) vb = p.B[(long)(b0 + row) * p.ldb + gk];
      }
      sa[k][row] = (double)va;
      sb[k][row] = (double)vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GR_BK; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = sa[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = sb[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  double* slot = p.part + ((long)bx * nks + ks) * (GR_T * GR_T);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4_f64 result layout: lane l, register r -> row l/16 + 4r
        int row = wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        int col = wn * 32 + j * 16 + (lane & 15);
        slot[row * GR_T + col] = acc[i][j][r];
      }
}

// block (tile, slice of 256 entries): sum the K slices in index order, write C (and the
// mirror for symmetric).
__device__ __forceinline__ void gram_reduce_body(const GramP& p, int bx, int by) {
  const int T = (p.L + GR_T - 1) / GR_T;
  int I, J;
  tile_of(bx, T, p.sym, I, J);
  const double* base = p.part + (long)bx * p.ksplit * (GR_T * GR_T);
  const int e = by * 256 + threadIdx.x;
  double s = 0.0;
  for (int k = 0; k < p.ksplit; ++k) s += base[(long)k * GR_T * GR_T + e];
  const int a = I * GR_T + e / GR_T, b = J * GR_T + e % GR_T;
  if (a < p.L && b < p.L) {
    if (!isfinite(s) && p.status) atomicOr(p.status, KFAC_DS_NONFINITE);
    p.C[(long)a * p.ldc + b] = s;
    if (p.sym && I != J) p.C[(long)b * p.ldc + a] = s;
  }
}

__global__ __launch_bounds__(256) void k_gram_partial(GramP p) { gram_partial_body(p, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(256) void k_gram_reduce(GramP p) { gram_reduce_body(p, blockIdx.x, blockIdx.y); }
KFAC_GROUPED_KERNEL(k_gram_partial_g, gram_partial_body, GramP, 256)
KFAC_GROUPED_KERNEL(k_gram_reduce_g, gram_reduce_body, GramP, 256)

// ======================================================================================
// Cholesky of the l x l Gram (one workgroup of 512 threads), nb = 16 blocks.
//   W  <- G (+ shift I on the retry), lower part overwritten by L (G = L L^T)
//   Li <- inverses of the 16 x 16 diagonal blocks of L (row-major, identity-padded)
// The shift follows shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yamazaki
// 2020): s = 11 (m l + l (l + 1)) u ||Y||_2^2, with ||Y||_2^2 bounded by trace(G).
// ======================================================================================
constexpr int CH_NB = 16;
constexpr int CH_MAXN = KFAC_MAX_SKETCH;

__global__ __launch_bounds__(512) void k_cholesky(const double* G, long ldg, int n, long m_rows,
                                                   double* W, long ldw, double* Li, int* status,
                                                   int* fail_flag) {
  __shared__ double P[CH_MAXN - CH_NB][CH_NB + 1];   // panel L21
  __shared__ double Lbi[CH_NB][CH_NB + 1];           // inverse of the diagonal block
  __shared__ int sfail;
  __shared__ double strace;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (n + CH_NB - 1) / CH_NB;

  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += G[(long)i * ldg + i];
    strace = t;
  }
  __syncthreads();
  const double shift = 11.0 * ((double)m_rows * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * strace;

  for (int attempt = 0; attempt < 2; ++attempt) {
    // W <- G (+ shift I)
    for (long e = tid; e < (long)n * n; e += blockDim.x) {
      int i = (int)(e / n), j = (int)(e % n);
      double v = G[(long)i * ldg + j];
      if (attempt == 1 && i == j) v += shift;
      W[(long)i * ldw + j] = v;
    }
    if (tid == 0) sfail = 0;
    __syncthreads();

    for (int b = 0; b < nblk; ++b) {
      const int kb = b * CH_NB;
      const int nbk = min(CH_NB, n - kb);
      // ---- (1) diagonal block: wave 0, lane i < 16 owns row i ------------------------
      if (wave == 0) {
        double row[CH_NB];
        const int i = lane & (CH_NB - 1);
_Pragma("clang loop unroll(full)")
        for (int j = 0; j < CH_NB; ++j) {
          double v = (i == j) ? 1.0 : 0.0;
          if (i < nbk && j < nbk) v = W[(long)(kb + i) * ldw + kb + j];
          row[j] = v;
        }
        bool fail = false;
_Pragma("clang loop unroll(full)")
        for (int j = 0; j < CH_NB; ++j) {
          double piv = __shfl(row[j], j, 64);
          if (!(piv > 0.0) || !isfinite(piv)) { fail = true; piv = 1.0; }
          double ljj = sqrt(piv);
          if (i == j) row[j] = ljj;
          else if (i > j) row[j] = row[j] / ljj;
_Pragma("clang loop unroll(full)")
          for (int k = j + 1; k < CH_NB; ++k) {
            double lkj = __shfl(row[j], k, 64);
            if (i >= k) row[k] -= row[j] * lkj;
          }
        }
        // inverse X = L^{-1} of the lower-triangular block, right-looking: lane i keeps
        // row i of X; column j is finalised row by row (X[s][j] = y_s / L[s][s], then
        // y_i -= L[i][s] X[s][j] for i > s), so every shuffle depends on the previous step.
        double xc[CH_NB];
        _Pragma("clang loop unroll(full)")
        for (int j = 0; j < CH_NB; ++j) xc[j] = (i == j) ? 1.0 : 0.0;
        _Pragma("clang loop unroll(full)")
        for (int j = 0; j < CH_NB; ++j) {
          _Pragma("clang loop unroll(full)")
          for (int sr = j; sr < CH_NB; ++sr) {
            if (i == sr) xc[j] = xc[j] / row[sr];
            const double xs = __shfl(xc[j], sr, 64);
            if (i > sr) xc[j] -= row[sr] * xs;
          }
        }
        if (lane < CH_NB) {
          _Pragma("clang loop unroll(full)")
          for (int j = 0; j < CH_NB; ++j) {
            if (i < nbk && j <= i) W[(long)(kb + i) * ldw + kb + j] = row[j];
            Lbi[i][j] = xc[j];
            Li[(long)b * CH_NB * CH_NB + i * CH_NB + j] = xc[j];
          }
        }
        if (fail && lane == 0) sfail = 1;
      }
      __syncthreads();
      if (sfail) break;
      // ---- (2) panel: L21[i][:] = G21[i][:] * Lbb^{-T} -------------------------------
      const int m = n - kb - CH_NB;   // rows below the block
      for (int i = tid; i < m; i += blockDim.x) {
        double out[CH_NB];
#pragma unroll
        for (int t = 0; t < CH_NB; ++t) out[t] = 0.0;
        const double* wrow = W + (long)(kb + CH_NB + i) * ldw + kb;
#pragma unroll 1
        for (int sidx = 0; sidx < CH_NB; ++sidx) {   // Lbi is lower triangular
          const double gs = wrow[sidx];
#pragma unroll
          for (int t = 0; t < CH_NB; ++t) out[t] += gs * Lbi[t][sidx];
        }
#pragma unroll
        for (int t = 0; t < CH_NB; ++t) {
          P[i][t] = out[t];
          W[(long)(kb + CH_NB + i) * ldw + kb + t] = out[t];
        }
      }
      __syncthreads();
      // ---- (3) trailing update, lower triangle: W22[i][k] -= P[i] . P[k] ------------
      if (m > 0) {
        long cnt = (long)m * (m + 1) / 2;
        for (long e = tid; e < cnt; e += blockDim.x) {
          // e -> (i, k) with k <= i, row-major over the packed lower triangle
          int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
          while ((long)i * (i + 1) / 2 > e) --i;
          while ((long)(i + 1) * (i + 2) / 2 <= e) ++i;
          int k = (int)(e - (long)i * (i + 1) / 2);
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < CH_NB; ++t) acc += P[i][t] * P[k][t];
          W[(long)(kb + CH_NB + i) * ldw + kb + CH_NB + k] -= acc;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    if (!sfail) break;
    if (tid == 0) atomicOr(status, attempt == 0 ? KFAC_DS_CHOL_SHIFTED : KFAC_DS_CHOL_FAILED);
    __syncthreads();
  }
  if (tid == 0) *fail_flag = sfail;
}

// ======================================================================================
// Forward substitution Q^T = L^{-1} Y^T, NC columns of Y^T per workgroup (256 threads):
// for each 16-row block b:  X_b = Li_b (Y_b - L_{b,<b} X_{<b}); the block row of L is
// staged in LDS.  fp64 arithmetic, fp32 (and optional bf16) output, rows >= n zero.
// ======================================================================================
template <int NMAX, int NC>
__global__ __launch_bounds__(256) void k_trsm(const double* W, long ldw, const double* Li, int n, int l_pad,
                                              const float* Yt, long ldy, int ncols, float* Qt, long ldq,
                                              uint16_t* Qtb, long ldqb) {
  __shared__ double X[NMAX][NC + 1];
  __shared__ double Lr[CH_NB][NMAX + 1];
  __shared__ double Lib[CH_NB][CH_NB + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * NC;
  const int nblk = (n + CH_NB - 1) / CH_NB;
  for (int e = tid; e < nblk * CH_NB * NC; e += 256) {
    const int i = e / NC, c = e % NC;
    double v = 0.0;
    if (i < n && c0 + c < ncols) v = (double)Yt[(long)i * ldy + c0 + c];
    X[i][c] = v;
  }
  constexpr int CPT = CH_NB * NC / 256;           // columns per thread
  const int il = tid / (NC / CPT), cq = (tid % (NC / CPT)) * CPT;
  for (int b = 0; b < nblk; ++b) {
    const int kb = b * CH_NB;
    for (int e = tid; e < CH_NB * kb; e += 256) {
      const int rr = e / kb, ss = e % kb;
      Lr[rr][ss] = (kb + rr < n) ? W[(long)(kb + rr) * ldw + ss] : 0.0;
    }
    {
      const int rr = tid / CH_NB, ss = tid % CH_NB;
      Lib[rr][ss] = Li[(long)b * CH_NB * CH_NB + tid];
    }
    __syncthreads();
    const int i = kb + il;
    double t[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) t[u] = X[i][cq + u];
    for (int sidx = 0; sidx < kb; ++sidx) {
      const double l = Lr[il][sidx];
#pragma unroll
      for (int u = 0; u < CPT; ++u) t[u] -= l * X[sidx][cq + u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CPT; ++u) X[i][cq + u] = t[u];
    __syncthreads();
    double o[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) o[u] = 0.0;
#pragma unroll
    for (int sidx = 0; sidx < CH_NB; ++sidx) {
      const double l = Lib[il][sidx];
#pragma unroll
      for (int u = 0; u < CPT; ++u) o[u] += l * X[kb + sidx][cq + u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CPT; ++u) X[i][cq + u] = (i < n) ? o[u] : 0.0;
    __syncthreads();
  }
  for (int e = tid; e < l_pad * NC; e += 256) {
    const int i = e / NC, c = e % NC;
    if (c0 + c >= ncols) continue;
    const float v = (i < n) ? (float)X[i][c] : 0.f;
    Qt[(long)i * ldq + c0 + c] = v;
    if (Qtb) Qtb[(long)i * ldqb + c0 + c] = f32_to_bf16_rne(v);
  }
}

// ======================================================================================
// Register-resident Cholesky for n <= 288 (1024 threads; same 32 x 32 thread grid and
// 9 x 9 blocks of 32 as the tridiagonalisation).  Right-looking, one column per step:
// the pivot owner publishes a_kk, the owners of column k scale it (l_ik = a_ik / l_kk,
// written to W and LDS), every thread applies a_ij -= l_ik l_jk to its active slots.
// Retried once with the shifted-CholeskyQR shift.  Afterwards the 16 x 16 diagonal
// blocks of L are inverted in parallel (one wavefront per block) into Li.
// ======================================================================================
constexpr int RB = 32, RNB = 9, RNMAX = RB * RNB;

__device__ __forceinline__ constexpr int rslot(int I, int J) { return I * (I + 1) / 2 + J; }

__device__ void invert_diag_blocks(const double* W, long ldw, int n, double* Li) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nblk = (n + CH_NB - 1) / CH_NB;
  const int i = lane & (CH_NB - 1);
  for (int b = wave; b < nblk; b += nw) {
    const int kb = b * CH_NB, nbk = min(CH_NB, n - kb);
    double row[CH_NB];
    _Pragma("clang loop unroll(full)")
    for (int j = 0; j < CH_NB; ++j) {
      double v = (i == j) ? 1.0 : 0.0;
      if (i < nbk && j < nbk && j <= i) v = W[(long)(kb + i) * ldw + kb + j];
      row[j] = v;
    }
    double xc[CH_NB];
    _Pragma("clang loop unroll(full)")
    for (int j = 0; j < CH_NB; ++j) xc[j] = (i == j) ? 1.0 : 0.0;
    _Pragma("clang loop unroll(full)")
    for (int j = 0; j < CH_NB; ++j) {
      _Pragma("clang loop unroll(full)")
      for (int sr = j; sr < CH_NB; ++sr) {
        if (i == sr) xc[j] = xc[j] / row[sr];
        const double xs = __shfl(xc[j], sr, 64);
        if (i > sr) xc[j] -= row[sr] * xs;
      }
    }
    if (lane < CH_NB) {
      _Pragma("clang loop unroll(full)")
      for (int j = 0; j < CH_NB; ++j) Li[(long)b * CH_NB * CH_NB + i * CH_NB + j] = xc[j];
    }
  }
}

__global__ __launch_bounds__(1024) void k_cholesky_reg(const double* G, long ldg, int n, long m_rows, double* W,
                                                       long ldw, double* Li, int* status, int* fail_flag) {
  __shared__ double scol[RNMAX];
  __shared__ double spiv;
  __shared__ double strace;
  __shared__ int sfail;
  const int t = threadIdx.x, tr = t >> 5, tc = t & 31, lane = t & 63, wave = t >> 6;
  if (wave == 0) {
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += G[(long)i * ldg + i];
    s = wave_sum(s);
    if (lane == 0) strace = s;
  }
  __syncthreads();
  const double shift = 11.0 * ((double)m_rows * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * strace;
  double a[45];
  int failed = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
#pragma unroll
    for (int I = 0; I < RNB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int i = RB * I + tr, j = RB * J + tc;
        double v = 0.0;
        if (i < n && j < n && (I != J || tr >= tc)) {
          v = G[(long)i * ldg + j];
          if (attempt == 1 && i == j) v += shift;
        }
        a[rslot(I, J)] = v;
      }
    if (t == 0) { spiv = a[0]; sfail = 0; }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const double piv = spiv;
      if (!(piv > 0.0) || !isfinite(piv)) { if (t == 0) sfail = 1; break; }   // uniform
      const double lkk = sqrt(piv), inv = 1.0 / lkk;
      const int J0 = k >> 5, c0 = k & 31;
      if (tc == c0) {
#pragma unroll
        for (int I = 0; I < RNB; ++I)
#pragma unroll
          for (int J = 0; J <= I; ++J)
            if (J == J0) {
              const int i = RB * I + tr;
              if (i == k) {
                a[rslot(I, J)] = lkk;
                W[(long)k * ldw + k] = lkk;
              } else if (i > k && i < n) {
                const double l = a[rslot(I, J)] * inv;
                a[rslot(I, J)] = l;
                scol[i] = l;
                W[(long)i * ldw + k] = l;
              }
            }
      }
      __syncthreads();
      const int kb = (k + 1) >> 5;
#pragma unroll
      for (int J = 0; J < RNB; ++J) {
        if (J >= kb) {
          const int j = RB * J + tc;
          const double lj = (j > k && j < n) ? scol[j] : 0.0;
#pragma unroll
          for (int I = J; I < RNB; ++I) {
            const int i = RB * I + tr;
            const double li = (i > k && i < n) ? scol[i] : 0.0;
            if (I != J || tr >= tc) a[rslot(I, J)] -= li * lj;
          }
        }
      }
      // publish the next pivot
      const int k1 = k + 1;
      if (k1 < n && tr == (k1 & 31) && tc == (k1 & 31)) {
#pragma unroll
        for (int I = 0; I < RNB; ++I)
          if (I == (k1 >> 5)) spiv = a[rslot(I, I)];
      }
      __syncthreads();
    }
    __syncthreads();
    failed = sfail;
    if (!failed) break;
    if (t == 0) atomicOr(status, attempt == 0 ? KFAC_DS_CHOL_SHIFTED : KFAC_DS_CHOL_FAILED);
    __syncthreads();
  }
  if (t == 0) *fail_flag = failed;
  __syncthreads();
  invert_diag_blocks(W, ldw, n, Li);
}

// ======================================================================================
// Fused Cholesky and inverse for n <= 288 (one workgroup of 1024 threads):
//   G = L L^T  and  X = L^{-1}, computed in place in one lower triangle M.
// Right-looking over k: with l_kk = sqrt(M_kk),
//   column k (rows i > k):  l_ik = M_ik / l_kk,   M_ik <- -l_ik / l_kk      (= X_ik)
//   row k (cols j < k):     M_kj <- M_kj / l_kk (= X_kj),   M_kk <- 1 / l_kk
//   rows i > k, j != k:     M_ij -= l_ik u_j,  u_j = l_jk (j > k) or X_kj (j < k)
// so columns > k hold the trailing Cholesky matrix and columns <= k hold the rows of
// L^{-1} built by forward substitution of L X = I.  Thread grid 32 x 32 over 9 x 9
// blocks of 32: off-diagonal blocks in registers, diagonal blocks in LDS.  Retried
// once with the shifted-CholeskyQR shift.  Output Linv (l_pad x l_pad, zero above the
// diagonal and outside n x n).
// ======================================================================================
constexpr int CB = 32, CNB = 9, CNMAX = CB * CNB;

__device__ __forceinline__ constexpr int oslot(int I, int J) { return I * (I - 1) / 2 + J; }   // I > J

struct CholSh {
  double (*Ld)[CB][CB + 1];
  double* sl;
  double* su;
  double* spiv;
  int* sfail;
};

// Columns k = 32 K0 + c0 of block column K0 (compile-time).
template <int K0>
__device__ __forceinline__ void cholinv_block_col(double (&a)[36], const CholSh& S, int n) {
  const int t = threadIdx.x, tr = t >> 5, tc = t & 31;
  double (*Ld)[CB][CB + 1] = S.Ld;
  double* sl = S.sl;
  double* su = S.su;
  if (CB * K0 >= n || *S.sfail) return;                    // uniform
  for (int c0 = 0; c0 < CB; ++c0) {
    const int k = CB * K0 + c0;
    if (k >= n) break;                                      // uniform
    const double piv = *S.spiv;
    if (!(piv > 0.0) || !isfinite(piv)) { if (t == 0) *S.sfail = 1; break; }   // uniform
    const double lkk = sqrt(piv), inv = 1.0 / lkk;
    // (A) column k below the diagonal (l_ik, then X_ik = -l_ik / l_kk) and row k
    if (tc == c0) {
      {
        const int i = CB * K0 + tr;
        if (i > k && i < n) { const double l = Ld[K0][tr][tc] * inv; sl[i] = l; Ld[K0][tr][tc] = -l * inv; }
      }
#pragma unroll
      for (int I = K0 + 1; I < CNB; ++I) {
        const int i = CB * I + tr;
        if (i < n) {
          const double l = a[oslot(I, K0)] * inv;
          sl[i] = l;
          a[oslot(I, K0)] = -l * inv;
        }
      }
    }
    if (tr == c0) {
#pragma unroll
      for (int J = 0; J < K0; ++J) {
        const double x = a[oslot(K0, J)] * inv;
        su[CB * J + tc] = x;
        a[oslot(K0, J)] = x;
      }
      const int j = CB * K0 + tc;
      if (j < k) { const double x = Ld[K0][tr][tc] * inv; su[j] = x; Ld[K0][tr][tc] = x; }
      else if (j == k) Ld[K0][tr][tc] = inv;
    }
    __syncthreads();
    // (B) rows i > k:  M_ij -= l_ik u_j,  u_j = l_jk (j > k) or X_kj (j < k), u_k = 0
#pragma unroll
    for (int I = K0; I < CNB; ++I) {
      const int i = CB * I + tr;
      const double li = (i > k && i < n) ? sl[i] : 0.0;
      {
        const int j = CB * I + tc;
        const double uj = (j > k && j < n) ? sl[j] : ((j < k) ? su[j] : 0.0);
        if (tr >= tc) Ld[I][tr][tc] -= li * uj;
      }
#pragma unroll
      for (int J = 0; J < I; ++J) {
        const int j = CB * J + tc;
        const double uj = (j > k && j < n) ? sl[j] : ((j < k) ? su[j] : 0.0);
        a[oslot(I, J)] -= li * uj;
      }
    }
    __syncthreads();
    const int k1 = k + 1;
    if (t == 0 && k1 < n) *S.spiv = Ld[k1 >> 5][k1 & 31][k1 & 31];
    __syncthreads();
  }
}

template <int... Ks>
__device__ __forceinline__ void cholinv_all_cols(std::integer_sequence<int, Ks...>, double (&a)[36],
                                                 const CholSh& S, int n) {
  (cholinv_block_col<Ks>(a, S, n), ...);
}

// attempt 0: plain Cholesky; attempt 1 (launched right after): returns at once unless
// attempt 0 broke down, else retries with the shifted-CholeskyQR shift.
__device__ __forceinline__ void cholinv_body(const CholInvTask& q, int, int) {
  const double* G = q.G; const long ldg = q.ldg; const int n = q.n; const long m_rows = q.m_rows;
  double* Linv = q.Linv; const long ldl = q.ldl; const int l_pad = q.l_pad;
  int* status = q.status; int* fail_flag = q.fail_flag; const int attempt = q.attempt;
  __shared__ double Ld[CNB][CB][CB + 1];
  __shared__ double sl[CNMAX];
  __shared__ double su[CNMAX];
  __shared__ double spiv;
  __shared__ double sshift;
  __shared__ int sfail;
  if (attempt == 1 && *fail_flag == 0) return;             // uniform
  const int t = threadIdx.x, tr = t >> 5, tc = t & 31, lane = t & 63, wave = t >> 6;
  if (attempt == 1) {
    if (wave == 0) {
      double sm = 0.0;
      for (int i = lane; i < n; i += 64) sm += G[(long)i * ldg + i];
      sm = wave_sum(sm);
      if (lane == 0) sshift = 11.0 * ((double)m_rows * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * sm;
    }
  } else if (t == 0) {
    sshift = 0.0;
  }
  __syncthreads();
  const double shift = sshift;
  double a[36];
#pragma unroll
  for (int I = 0; I < CNB; ++I) {
    const int i = CB * I + tr;
    {
      const int j = CB * I + tc;
      double v = 0.0;
      if (i < n && j < n && tr >= tc) {
        v = G[(long)i * ldg + j];
        if (i == j) v += shift;
      }
      Ld[I][tr][tc] = v;
    }
#pragma unroll
    for (int J = 0; J < I; ++J) {
      const int j = CB * J + tc;
      a[oslot(I, J)] = (i < n && j < n) ? G[(long)i * ldg + j] : 0.0;
    }
  }
  __syncthreads();
  if (t == 0) { spiv = Ld[0][0][0]; sfail = 0; }
  __syncthreads();
  const CholSh S{Ld, sl, su, &spiv, &sfail};
  cholinv_all_cols(std::make_integer_sequence<int, CNB>{}, a, S, n);
  __syncthreads();
  const int failed = sfail;
  if (t == 0) {
    *fail_flag = failed;
    if (failed) atomicOr(status, attempt == 0 ? KFAC_DS_CHOL_SHIFTED : KFAC_DS_CHOL_FAILED);
  }
  // write L^{-1} (lower), zeros elsewhere inside l_pad x l_pad
#pragma unroll
  for (int I = 0; I < CNB; ++I) {
    const int i = CB * I + tr;
    if (i >= l_pad) continue;
    double* row = Linv + (long)i * ldl;
    {
      const int j = CB * I + tc;
      if (j < l_pad) row[j] = (i < n && j < n && tr >= tc) ? Ld[I][tr][tc] : 0.0;
    }
#pragma unroll
    for (int J = 0; J < I; ++J) {
      const int j = CB * J + tc;
      if (j < l_pad) row[j] = (i < n && j < n) ? a[oslot(I, J)] : 0.0;
    }
#pragma unroll
    for (int J = I + 1; J < CNB; ++J) {
      const int j = CB * J + tc;
      if (j < l_pad) row[j] = 0.0;
    }
  }
}

__global__ __launch_bounds__(1024) void k_cholinv_reg(CholInvTask q) { cholinv_body(q, 0, 0); }
KFAC_GROUPED_KERNEL(k_cholinv_reg_g, cholinv_body, CholInvTask, 1024)

// ======================================================================================
// Q^T = L^{-1} Y^T on fp64 MFMA: L^{-1} (l_pad x l_pad fp64, lower), Y^T (l_pad x d fp32),
// output fp32 (and optional bf16).  Tile 64 (rows of Q^T) x 64 (columns), 4 waves of
// 32 x 32; the contraction stops at the tile's last row (triangular).
// grid (ceil(d/64), l_pad/64).
// ======================================================================================
__device__ __forceinline__ void trmm_body(const TrmmTask& q, int bx, int by) {
  const double* Li = q.Li; const long ldl = q.ldl; const int n = q.n;
  const float* Yt = q.Yt; const long ldy = q.ldy; const int ncols = q.ncols;
  float* Qt = q.Qt; const long ldq = q.ldq; uint16_t* Qtb = q.Qtb; const long ldqb = q.ldqb; const int l_pad = q.l_pad;
  __shared__ double sa[GR_BK][GR_T + 2];
  __shared__ double sb[GR_BK][GR_T + 2];
  const int a0 = by * GR_T, c0 = bx * GR_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
  const int kend = min(n, a0 + GR_T);
  for (int k0 = 0; k0 < kend; k0 += GR_BK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * 256;
      // A: 64 rows x 16 k (k contiguous in memory)
      {
        const int row = e / GR_BK, kk = e % GR_BK;
        double v = 0.0;
        if (a0 + row < n && k0 + kk < kend) v = Li[(long)(a0 + row) * ldl + k0 + kk];
        sa[kk][row] = v;
      }
      // B: 16 k x 64 columns (columns contiguous)
      {
        const int kk = e / GR_T, col = e % GR_T;
        double v = 0.0;
        if (k0 + kk < kend && c0 + col < ncols) v = (double)Yt[(long)(k0 + kk) * ldy + c0 + col];
        sb[kk][col] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GR_BK; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = sa[kk + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = sb[kk + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = a0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;   // f64 MFMA result layout
        const int col = c0 + wn * 32 + j * 16 + (lane & 15);
        if (row < l_pad && col < ncols) {
          const float v = (row < n) ? (float)acc[i][j][r] : 0.f;
          Qt[(long)row * ldq + col] = v;
          if (Qtb) Qtb[(long)row * ldqb + col] = f32_to_bf16_rne(v);
        }
      }
}

__global__ __launch_bounds__(256) void k_trmm_f64(TrmmTask q) { trmm_body(q, blockIdx.x, blockIdx.y); }
KFAC_GROUPED_KERNEL(k_trmm_f64_g, trmm_body, TrmmTask, 256)

// ======================================================================================
// Host launchers
// ======================================================================================
int gram_ksplit(int L, int K, int sym) {
  int T = (L + GR_T - 1) / GR_T;
  int tiles = sym ? T * (T + 1) / 2 : T * T;
  int want = (512 + tiles - 1) / tiles;
  int maxk = (K + 255) / 256;
  int ks = want < maxk ? want : maxk;
  if (ks < 1) ks = 1;
  if (ks > 128) ks = 128;
  return ks;
}

size_t gram_workspace_bytes(int L, int K, int sym) {
  int T = (L + GR_T - 1) / GR_T;
  int tiles = sym ? T * (T + 1) / 2 : T * T;
  return (size_t)tiles * gram_ksplit(L, K, sym) * GR_T * GR_T * sizeof(double);
}

GramP make_gram_task(const float* A, long lda, const float* B, long ldb, int L, int K, int sym, double* part,
                     double* C, long ldc, int* status) {
  GramP p{A, lda, B, ldb, L, K, sym, gram_ksplit(L, K, sym), part, C, ldc, status};
  return p;
}
int gram_tiles(int L, int sym) {
  const int T = (L + GR_T - 1) / GR_T;
  return sym ? T * (T + 1) / 2 : T * T;
}

hipError_t launch_gram(const float* A, long lda, const float* B, long ldb, int L, int K, int sym,
                       double* part, double* C, long ldc, int* status, hipStream_t s) {
  GramP p = make_gram_task(A, lda, B, ldb, L, K, sym, part, C, ldc, status);
  int T = (L + GR_T - 1) / GR_T;
  int tiles = sym ? T * (T + 1) / 2 : T * T;
  hipLaunchKernelGGL(k_gram_partial, dim3(tiles, p.ksplit), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_gram_reduce, dim3(tiles, GR_T * GR_T / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* G, long ldg, int n, long m_rows, double* W, long ldw, double* Li,
                           int* status, int* fail_flag, hipStream_t s) {
  if (n <= RNMAX)
    hipLaunchKernelGGL(k_cholesky_reg, dim3(1), dim3(1024), 0, s, G, ldg, n, m_rows, W, ldw, Li, status, fail_flag);
  else
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(512), 0, s, G, ldg, n, m_rows, W, ldw, Li, status, fail_flag);
  return hipGetLastError();
}

hipError_t launch_cholinv(const double* G, long ldg, int n, long m_rows, double* Linv, long ldl, int l_pad,
                          int* status, int* fail_flag, hipStream_t s) {
  CholInvTask q{G, ldg, n, m_rows, Linv, ldl, l_pad, status, fail_flag, 0};
  hipLaunchKernelGGL(k_cholinv_reg, dim3(1), dim3(1024), 0, s, q);
  q.attempt = 1;
  hipLaunchKernelGGL(k_cholinv_reg, dim3(1), dim3(1024), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* Li, long ldl, int n, const float* Yt, long ldy, int ncols, float* Qt, long ldq,
                       uint16_t* Qtb, long ldqb, int l_pad, hipStream_t s) {
  TrmmTask q{Li, ldl, n, Yt, ldy, ncols, Qt, ldq, Qtb, ldqb, l_pad};
  dim3 grid((ncols + GR_T - 1) / GR_T, (l_pad + GR_T - 1) / GR_T);
  hipLaunchKernelGGL(k_trmm_f64, grid, dim3(256), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_trsm(const double* W, long ldw, const double* Li, int n, int l_pad, const float* Yt, long ldy,
                       int ncols, float* Qt, long ldq, uint16_t* Qtb, long ldqb, hipStream_t s) {
  if (n <= 288) {
    hipLaunchKernelGGL((k_trsm<288, 32>), dim3((ncols + 31) / 32), dim3(256), 0, s, W, ldw, Li, n, l_pad, Yt,
                       ldy, ncols, Qt, ldq, Qtb, ldqb);
  } else {
    hipLaunchKernelGGL((k_trsm<CH_MAXN, 16>), dim3((ncols + 15) / 16), dim3(256), 0, s, W, ldw, Li, n, l_pad,
                       Yt, ldy, ncols, Qt, ldq, Qtb, ldqb);
  }
  return hipGetLastError();
}

#define KFAC_GLAUNCH(FN, KER, T, NT)                                                         \
  hipError_t FN(const T* tasks, GroupMap gm, int blocks, hipStream_t s) {                  \
    if (blocks > 0) hipLaunchKernelGGL(KER, dim3(blocks), dim3(NT), 0, s, tasks, gm);      \
    return hipGetLastError();                                                              \
  }
KFAC_GLAUNCH(launch_gram_partial_g, k_gram_partial_g, GramP, 256)
KFAC_GLAUNCH(launch_gram_reduce_g, k_gram_reduce_g, GramP, 256)
KFAC_GLAUNCH(launch_cholinv_g, k_cholinv_reg_g, CholInvTask, 1024)
KFAC_GLAUNCH(launch_trmm_g, k_trmm_f64_g, TrmmTask, 256)
int gram_reduce_slices() { return GR_T * GR_T / 256; }
int trmm_blocks_x(int ncols) { return (ncols + GR_T - 1) / GR_T; }
int trmm_blocks_y(int l_pad) { return (l_pad + GR_T - 1) / GR_T; }
}  // namespace kfac
