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
constexpr int GR_T = 64;

__device__ __forceinline__ void tile_of(int t, int T, int sym, int& I, int& J) {
  if (sym) { upper_tile(t, T, I, J); }
  else { I = t / T; J = t % T; }
}

// block (tile, K slice), 256 threads = 2 x 2 waves of 32 x 32, 32-wide K steps.  The
// next step's operands are loaded into registers (16-byte row loads when the rows are
// 16-byte aligned) while the MFMAs run on the current one.
constexpr int GP_BK = 32;
__device__ __forceinline__ void gram_partial_body(const GramP& p, int bx, int by) {
  __shared__ double sa[GP_BK][GR_T + 2];
  __shared__ double sb[GP_BK][GR_T + 2];
  const int T = (p.L + GR_T - 1) / GR_T;
  int I, J;
  tile_of(bx, T, p.sym, I, J);
  const int a0 = I * GR_T, b0 = J * GR_T;
  const int ks = by, nks = p.ksplit;
  const int kchunk = ((p.K + nks - 1) / nks + GP_BK - 1) / GP_BK * GP_BK;
  const int kb = ks * kchunk, ke = min(p.K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // loader: thread -> rows lr and lr + 32, k lk .. lk + 3 of the step
  const int lr = tid >> 3, lk = (tid & 7) * 4;
  const bool vec = ((p.lda & 3) == 0) && ((p.ldb & 3) == 0) && ((((uintptr_t)p.A) & 15) == 0) &&
                   ((((uintptr_t)p.B) & 15) == 0);
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
  float4 ra[2], rb[2];
  auto load_row = [&](const float* X, long ldx, int r0, int k0, int u) {
    const int row = r0 + lr + 32 * u, gk = k0 + lk;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < p.L) {
      const float* q = X + (long)row * ldx + gk;
      if (vec && gk + 4 <= ke) {
        v = *(const float4*)q;
      } else {
        if (gk + 0 < ke) v.x = q[0];
        if (gk + 1 < ke) v.y = q[1];
        if (gk + 2 < ke) v.z = q[2];
        if (gk + 3 < ke) v.w = q[3];
      }
    }
    return v;
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ra[u] = load_row(p.A, p.lda, a0, k0, u);
      rb[u] = load_row(p.B, p.ldb, b0, k0, u);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = lr + 32 * u;
      sa[lk + 0][row] = (double)ra[u].x; sa[lk + 1][row] = (double)ra[u].y;
      sa[lk + 2][row] = (double)ra[u].z; sa[lk + 3][row] = (double)ra[u].w;
      sb[lk + 0][row] = (double)rb[u].x; sb[lk + 1][row] = (double)rb[u].y;
      sb[lk + 2][row] = (double)rb[u].z; sb[lk + 3][row] = (double)rb[u].w;
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += GP_BK) {
    __syncthreads();                                 // the previous step's reads are done
    store();
    __syncthreads();
    if (k0 + GP_BK < ke) load(k0 + GP_BK);           // in flight during the MFMAs
#pragma unroll
    for (int kk = 0; kk < GP_BK; kk += 4) {
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
// Blocked Cholesky and inverse for l_pad <= 288.
// Launch 1 (k_cholinv, one workgroup of 512 threads per Gram, run as attempt 0 and then
// attempt 1 = shifted retry only where attempt 0 broke down):
//   G = L L^T, right-looking over 16-wide block columns K, with the trailing matrix on chip
//   for the whole factorisation: the strictly lower 16 x 16 tiles (I > J) in the registers of
//   wavefronts 1-7 (tile t = I (I - 1) / 2 + J in slot t / 7 of wavefront 1 + t mod 7, MFMA
//   accumulator layout), the diagonal tiles in LDS.  Per block column K, two barriers:
//   (a) panel: the owners of the tiles (I, K), I > K, form L_IK = A_IK X_KK^T (fp64 MFMA;
//       X_KK = L_KK^{-1} from LDS) into the LDS panel and the output;
//   (b) update: A_IJ -= L_IK L_JK^T for I >= J > K, operands from the panel.  Look-ahead:
//       wavefront 0 updates the next diagonal tile first and factors it (block K + 1) while
//       the others update the rest, the other diagonal tiles included.
//   The diagonal block is factored by one wavefront (element (r, c) of the symmetric block in
//   lane c, register r; pivots and columns by readlane) and inverted the same way; X_KK goes
//   to the output.  L overwrites the lower triangle of G (the strict upper triangle and a
//   saved copy of the diagonal keep G for the retry).
// Launch 2 (k_trtri_cols, one workgroup per (Gram, block column K)): the off-diagonal
//   blocks of X = L^{-1} down column K, X_IK = -X_II sum_{J=K}^{I-1} L_IJ X_JK, with the
//   column panel of X in LDS.
// Rows and columns >= n are treated as identity (and are zero in X).  The shift follows
// shifted CholeskyQR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yamazaki 2020):
// s = 11 (m l + l (l + 1)) u ||Y||_2^2, with ||Y||_2^2 bounded by trace(G).
// Output X (l_pad x l_pad, zero above the diagonal and outside n x n).
// ======================================================================================
constexpr int BC = 16, BC_NT = 512, TT_NT = 256;
constexpr int BC_NB = kCholInvMax / BC;                       // block rows at most
constexpr int BC_TW = BC_NT / 64 - 1;                         // wavefronts holding tiles
constexpr int BC_SLOTS = (BC_NB * (BC_NB - 1) / 2 + BC_TW - 1) / BC_TW;
static_assert(BC == 16 && kCholInvMax % BC == 0, "block shape");

struct BcSmem {
  double P[kCholInvMax][BC + 1];  // panel of block column K: A_IK, then L_IK (absolute rows)
  double D[BC_NB][BC][BC + 1];    // diagonal tiles (current values of the trailing matrix)
  double X[2][BC][BC + 1];        // inverse of the diagonal block K (buffer K mod 2)
  double shift;
  int fail;
};

// The diagonal block K (wavefront 0 only).  Lane c (c = lane mod 16) holds the whole column c of
// the symmetric block, so the multiplier l_cj of its own column is its own entry j; the
// pivot and column j come from lane j by readlane (uniform values, no LDS round trip).
// X = L_KK^{-1} follows by forward substitution on the columns of the identity (lane c:
// column c of X) with the columns of L broadcast the same way.  The lane index fed to
// each step's readlanes is passed through an empty asm that depends on the previous step,
// so the broadcasts are issued step by step (hoisted, they would all be live at once).
// The block's current values come from src (element (r, c) at src[r lds + c], lower
// triangle read).  Rows / columns >= n are identity.  Returns false on a non-positive or
// non-finite pivot.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ bool bc_diag_block(double* G, long ldg, int n, int K, double* Xo, long ldx,
                                              double (*Xs)[BC + 1], const double* src, long lds) {
  static_assert(BC == 16, "one lane per column of the diagonal block");
  // The lane split goes through an opaque move so that lane-dependent predicates and
  // constants are recomputed at each call instead of being hoisted out of the caller's
  // loop over K (hoisted, they stay live across the factorisation and spill).
  int lane, c;
  asm volatile("v_and_b32 %0, 63, %1" : "=v"(lane) : "v"((int)threadIdx.x));
  asm volatile("v_and_b32 %0, 15, %1" : "=v"(c) : "v"(lane));
  const int k0 = K * BC;
  const bool cin = k0 + c < n;
  double d[BC];
#pragma unroll
  for (int r = 0; r < BC; ++r) {
    const int hi = r > c ? r : c, lo = r > c ? c : r;   // the lower-triangle copy of (r, c)
    double v = (r == c) ? 1.0 : 0.0;
    if (cin && k0 + r < n) v = src[(long)hi * lds + lo];
    d[r] = v;
  }
  bool ok = true;
  double chain = 0.0;
  double rdiag[BC];
#pragma unroll
  for (int j = 0; j < BC; ++j) {
    int src = j;
    asm volatile("" : "+s"(src) : "v"(chain));
    const double piv = readlane_f64(d[j], src);
    ok = ok && piv > 0.0 && isfinite(piv);              // no early exit: one straight path
    const double inv = rsqrt_nr(piv), ljj = piv * inv;
    rdiag[j] = inv;
    const double lc = (c > j) ? d[j] * inv : 0.0;       // l_cj (c > j); 0 leaves columns < j
#pragma unroll
    for (int r = j + 1; r < BC; ++r) {
      const double lr = readlane_f64(d[r], src) * inv;  // column j of L
      d[r] = (c == j) ? lr : d[r] - lr * lc;
    }
    if (c == j) d[j] = ljj;
    chain = inv;
  }
  if (!ok) return false;
  // X = L^{-1}: lane c solves L x = e_c
  double x[BC];
#pragma unroll
  for (int r = 0; r < BC; ++r) x[r] = (r == c) ? 1.0 : 0.0;
  double xk = 0.0;
#pragma unroll
  for (int k = 0; k < BC; ++k) {
    int src = k;
    asm volatile("" : "+s"(src) : "v"(xk));
    xk = x[k] * rdiag[k];
    x[k] = xk;
#pragma unroll
    for (int r = k + 1; r < BC; ++r) x[r] -= readlane_f64(d[r], src) * xk;
  }
  if (lane < BC) {
#pragma unroll
    for (int r = 0; r < BC; ++r) {
      const bool in = cin && k0 + r < n && r >= c;
      if (in) G[(long)(k0 + r) * ldg + k0 + c] = d[r];
      const double xr = in ? x[r] : 0.0;               // zero outside n x n
      Xo[(long)(k0 + r) * ldx + k0 + c] = xr;
      Xs[r][c] = xr;
    }
  }
  return true;
}

// Lower-triangle tile t of a T x T grid of tiles, row-major over I >= J (closed form; t
// is small, the float estimate is corrected by one step either way).
__device__ __forceinline__ void lower_tile(int t, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  if (i * (i + 1) / 2 > t) --i;
  if ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// Strictly lower tile t = I (I - 1) / 2 + J (I > J) of the block grid (closed form; t is
// small, the float estimate is corrected by one step either way).
__device__ __forceinline__ void strict_lower_tile(int t, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) + 1.0f) * 0.5f);
  if (i * (i - 1) / 2 > t) --i;
  if ((i + 1) * i / 2 <= t) ++i;
  I = i;
  J = t - i * (i - 1) / 2;
}

__device__ __forceinline__ void wg_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A -= P_I P_J^T on a 16 x 16 accumulator tile, operands from the LDS panel (rows of blocks I, J)
__device__ __forceinline__ f64x4 bc_update(f64x4 acc, const double (*P)[BC + 1], int I, int J, int lane) {
  double pa[BC / 4], pb[BC / 4];
#pragma unroll
  for (int u = 0; u < BC / 4; ++u) {
    const int kc = 4 * u + (lane >> 4);
    pa[u] = -P[I * BC + (lane & 15)][kc];
    pb[u] = P[J * BC + (lane & 15)][kc];
  }
#pragma unroll
  for (int u = 0; u < BC / 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[u], pb[u], acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ f64x4 bc_load_tile(const double (*T)[BC + 1], int lane) {
  f64x4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = T[(lane >> 4) + 4 * r][lane & 15];
  return a;
}
__device__ __forceinline__ void bc_store_tile(double (*T)[BC + 1], f64x4 a, int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) T[(lane >> 4) + 4 * r][lane & 15] = a[r];
}

__device__ __forceinline__ void cholinv_body(const CholInvTask& q, int, int) {
  double* G = q.G; const long ldg = q.ldg; const int n = q.n;
  double* X = q.Linv; const long ldx = q.ldl; const int l_pad = q.l_pad;
  __shared__ BcSmem sm;
  const int attempt = q.attempt;
  if (attempt == 1 && __builtin_amdgcn_readfirstlane(*q.fail_flag) == 0) return;   // uniform
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = BC_NT / 64;
  if (attempt == 0 && q.skip) {
    // second pass of CholeskyQR2: the first pass's basis is kept when its Gram is I to tol
    __shared__ int s_far;
    if (tid == 0) s_far = 0;
    __syncthreads();
    // lower triangle, a row per wave and a column per lane, the loads of several rows in
    // flight together (n <= kCholInvMax)
    bool far = false;
    constexpr int PERC = (kCholInvMax + 63) / 64;
#pragma unroll 3
    for (int i = wave; i < n; i += nw) {
      const double* row = G + (long)i * ldg;
#pragma unroll
      for (int u = 0; u < PERC; ++u) {
        const int j = lane + 64 * u;
        if (j <= i && !(fabs(row[j] - (i == j ? 1.0 : 0.0)) <= q.tol)) far = true;
      }
    }
    if (far) s_far = 1;                                       // benign race: same value
    __syncthreads();
    const bool keep = (s_far == 0);
    if (tid == 0) {
      *q.skip = keep ? 1 : 0;
      if (keep) *q.fail_flag = 0;
    }
    if (__builtin_amdgcn_readfirstlane(keep ? 1 : 0)) return;  // uniform
  }
  const int NB = l_pad / BC;
  // ---- set-up: save the diagonal (attempt 0) or restore G and shift it (attempt 1)
  if (attempt == 0) {
    for (int i = tid; i < n; i += BC_NT) q.dsave[i] = G[(long)i * ldg + i];
    if (tid == 0) sm.shift = 0.0;
  } else {
    for (int i = wave + 1; i < n; i += nw)                    // a row per wave: the lower part
      for (int j = lane; j < i; j += 64) G[(long)i * ldg + j] = G[(long)j * ldg + i];
    if (wave == 0) {
      double tr = 0.0;
      for (int i = lane; i < n; i += 64) tr += q.dsave[i];
      tr = wave_sum(tr);
      if (lane == 0) sm.shift = 11.0 * ((double)q.m_rows * n + (double)n * (n + 1)) * 1.1102230246251565e-16 * tr;
    }
    __syncthreads();
    for (int i = tid; i < n; i += BC_NT) G[(long)i * ldg + i] = q.dsave[i] + sm.shift;
  }
  if (tid == 0) sm.fail = 0;
  // zero the strict upper block triangle of the output, a row per wave
  for (int i = wave; i < l_pad; i += nw)
    for (int j = (i / BC + 1) * BC + lane; j < l_pad; j += 64) X[(long)i * ldx + j] = 0.0;
  // the diagonal tiles into LDS (identity outside n x n); G's global writes above are
  // visible to the whole workgroup after the barrier
  __syncthreads();
  for (int e = tid; e < NB * BC * BC; e += BC_NT) {
    const int J = e / (BC * BC), r = (e / BC) % BC, c = e % BC;
    const int i = J * BC + r, j = J * BC + c;
    sm.D[J][r][c] = (i < n && j < n) ? G[(long)i * ldg + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  // the two roles below run different code with the same barrier sequence (one barrier
  // after the set-up, then two per block column); the role and the loop exit are
  // wave-uniform (scalar) values, so every wavefront executes only its own role's barriers
  if (__builtin_amdgcn_readfirstlane(wave) == 0) {
    // ---- wavefront 0: the diagonal blocks, one step ahead of the panel
    if (!bc_diag_block(G, ldg, n, 0, X, ldx, sm.X[0], &sm.D[0][0][0], BC + 1) && lane == 0) sm.fail = 1;
    wg_barrier();                                             // X_00 and the flag visible
    for (int K = 0; K < NB; ++K) {
      if (__builtin_amdgcn_readfirstlane(sm.fail)) break;     // uniform over the workgroup
      wg_barrier();                                           // (a) panel L_.K in LDS
      if (K + 1 < NB) {
        f64x4 acc = bc_load_tile(sm.D[K + 1], lane);
        acc = bc_update(acc, sm.P, K + 1, K + 1, lane);
        bc_store_tile(sm.D[K + 1], acc, lane);
        wave_lds_order();
        if (!bc_diag_block(G, ldg, n, K + 1, X, ldx, sm.X[(K + 1) & 1], &sm.D[K + 1][0][0], BC + 1) && lane == 0)
          sm.fail = 1;
      }
      wg_barrier();                                           // (b) updates and X_K+1,K+1
    }
  } else {
    // ---- wavefronts 1-7: the strictly lower tiles in registers.  The block coordinates of
    // the slots are wave-uniform (scalar registers): slot sl holds tile (tI, tJ), tJ = -1 for
    // an empty slot
    const int tw = __builtin_amdgcn_readfirstlane(wave - 1);
    const int ntile = NB * (NB - 1) / 2;
    int tI[BC_SLOTS], tJ[BC_SLOTS];
#pragma unroll
    for (int sl = 0; sl < BC_SLOTS; ++sl) {
      const int t = tw + BC_TW * sl;
      int I = 0, J = -1;
      if (t < ntile) strict_lower_tile(t, I, J);
      tI[sl] = __builtin_amdgcn_readfirstlane(I);
      tJ[sl] = __builtin_amdgcn_readfirstlane(J);
    }
    f64x4 T[BC_SLOTS];
#pragma unroll
    for (int sl = 0; sl < BC_SLOTS; ++sl) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tI[sl] * BC + (lane >> 4) + 4 * r, col = tJ[sl] * BC + (lane & 15);
        T[sl][r] = (tJ[sl] >= 0 && row < n && col < n) ? G[(long)row * ldg + col] : 0.0;
      }
    }
    wg_barrier();                                             // X_00 visible
    for (int K = 0; K < NB; ++K) {
      if (__builtin_amdgcn_readfirstlane(sm.fail)) break;     // uniform over the workgroup
      const double (*Xk)[BC + 1] = sm.X[K & 1];
      // the lane index through an opaque move each step: lane-dependent addresses are then
      // formed where they are used instead of being hoisted for all slots at once (which
      // would hold them across the factorisation and spill)
      int lane;
      asm volatile("v_and_b32 %0, 63, %1" : "=v"(lane) : "v"((int)threadIdx.x));
      // (a) panel: L_IK = A_IK X_KK^T for the owned tiles (I, K): all of them staged into the
      // panel first (one LDS wait for all), then transformed
#pragma unroll
      for (int sl = 0; sl < BC_SLOTS; ++sl)
        if (tJ[sl] == K) bc_store_tile(&sm.P[tI[sl] * BC], T[sl], lane);   // uniform condition
      wave_lds_order();
#pragma unroll
      for (int sl = 0; sl < BC_SLOTS; ++sl) {
        const int I = tI[sl];
        if (tJ[sl] != K) continue;                            // uniform
        double a[BC / 4], b[BC / 4];
#pragma unroll
        for (int u = 0; u < BC / 4; ++u) {
          const int kc = 4 * u + (lane >> 4);
          a[u] = sm.P[I * BC + (lane & 15)][kc];
          b[u] = Xk[lane & 15][kc];
        }
        f64x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < BC / 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = I * BC + (lane >> 4) + 4 * r, col = K * BC + (lane & 15);
          const bool in = row < n && col < n;
          acc[r] = in ? acc[r] : 0.0;
          if (in) G[(long)row * ldg + col] = acc[r];
        }
        bc_store_tile(&sm.P[I * BC], acc, lane);
      }
      wg_barrier();                                           // (a) panel L_.K in LDS
      // (b) trailing update of the owned tiles and of the diagonal tiles J >= K + 2
#pragma unroll
      for (int sl = 0; sl < BC_SLOTS; ++sl) {
        if (tJ[sl] <= K) continue;                            // uniform (empty slots: -1)
        T[sl] = bc_update(T[sl], sm.P, tI[sl], tJ[sl], lane);
      }
      for (int J = K + 2 + tw; J < NB; J += BC_TW) {
        f64x4 acc = bc_load_tile(sm.D[J], lane);
        acc = bc_update(acc, sm.P, J, J, lane);
        bc_store_tile(sm.D[J], acc, lane);
      }
      wg_barrier();                                           // (b) updates and X_K+1,K+1
    }
  }
  if (tid == 0) {
    const int failed = sm.fail;
    *q.fail_flag = failed;
    if (failed) atomicOr(q.status, attempt == 0 ? KFAC_DS_CHOL_SHIFTED : KFAC_DS_CHOL_FAILED);
  }
}

__global__ __launch_bounds__(BC_NT) void k_cholinv(CholInvTask q) { cholinv_body(q, 0, 0); }
KFAC_GROUPED_KERNEL(k_cholinv_g, cholinv_body, CholInvTask, BC_NT)

// Launch 2: block column K = bx of X = L^{-1} below the diagonal.  For each block row
// I > K: T = L_I,[K, I) X_[K, I),K with the contraction split over the four wavefronts
// (partial tiles summed through LDS), then X_IK = -X_II T.
struct TtSmem {
  double Xc[288][BC + 1];         // X_JK for J >= K (absolute rows)
  double Tp[4][BC][BC + 1];       // per-wavefront partial T
  double Xd[BC][BC + 1];          // X_II
};

__device__ __forceinline__ void trtri_cols_body(const CholInvTask& q, int bx, int) {
  const double* L = q.G; const long ldg = q.ldg; const int n = q.n;
  double* X = q.Linv; const long ldx = q.ldl; const int l_pad = q.l_pad;
  __shared__ TtSmem sm;
  constexpr int CT = BC / 16, NTILE = CT * CT, KS = 4 / NTILE;   // tiles of T, contraction split
  static_assert(NTILE * KS == 4, "four wavefronts");
  const int NB = l_pad / BC, K = bx;
  if (K >= NB - 1) return;                                     // uniform
  if (q.skip && *q.skip) return;                               // pass kept (see cholinv)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k0 = K * BC;
  for (int e = tid; e < BC * BC; e += TT_NT) sm.Xc[k0 + e / BC][e % BC] = X[(long)(k0 + e / BC) * ldx + k0 + e % BC];
  const int tile = wave % NTILE, ks = wave / NTILE;
  const int rt = tile % CT, ct = tile / CT;
  // block row I's operands are loaded into registers one step ahead, while the MFMAs of
  // the previous row run: L_I,[K, I) straight in the MFMA operand layout (wavefront ks
  // takes the k-steps 4 ks + 16 m), and one element of X_II per thread
  static_assert(CT == 1 && KS == 4, "one 16 x 16 tile, four contraction slices");
  constexpr int NMK = 288 / 16;
  static_assert(BC * BC == TT_NT, "one element of X_II per thread");
  double ra[NMK], rx = 0.0;
  auto load = [&](int I) {
    const int i0 = I * BC, w = i0 - k0, row = i0 + (lane & 15);
#pragma unroll
    for (int m = 0; m < NMK; ++m) {
      const int kk = 4 * ks + 16 * m, col = k0 + kk + (lane >> 4);
      ra[m] = (kk < w && row < n && col < n) ? L[(long)row * ldg + col] : 0.0;
    }
    rx = X[(long)(i0 + tid / BC) * ldx + i0 + tid % BC];
  };
  if (K + 1 < NB) load(K + 1);
  __syncthreads();                                             // X_KK in Xc
  for (int I = K + 1; I < NB; ++I) {
    const int i0 = I * BC, w = i0 - k0;
    double a[NMK];
#pragma unroll
    for (int m = 0; m < NMK; ++m) a[m] = ra[m];
    sm.Xd[tid / BC][tid % BC] = rx;
    if (I + 1 < NB) load(I + 1);
    {
      f64x4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < NMK; ++m) {
        const int kk = 4 * ks + 16 * m;
        if (kk < w)                                            // uniform
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], sm.Xc[k0 + kk + (lane >> 4)][lane & 15], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) sm.Tp[ks][(lane >> 4) + 4 * r][lane & 15] = acc[r];
    }
    __syncthreads();
    if (KS > 1) {
      for (int e = tid; e < BC * BC; e += TT_NT) {
        double v = 0.0;
        for (int u = 0; u < KS; ++u) v += sm.Tp[u][e / BC][e % BC];
        sm.Tp[0][e / BC][e % BC] = v;
      }
      __syncthreads();
    }
    // X_IK = -X_II T
    if (wave < NTILE) {
      f64x4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < BC; kk += 4) {
        const int kc = kk + (lane >> 4);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-sm.Xd[rt * 16 + (lane & 15)][kc], sm.Tp[0][kc][ct * 16 + (lane & 15)],
                                                   acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + (lane >> 4) + 4 * r, col = ct * 16 + (lane & 15);
        const double v = (i0 + row < n && k0 + col < n) ? acc[r] : 0.0;
        sm.Xc[i0 + row][col] = v;
        X[(long)(i0 + row) * ldx + k0 + col] = v;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(TT_NT) void k_trtri_cols(CholInvTask q) { trtri_cols_body(q, blockIdx.x, 0); }
KFAC_GROUPED_KERNEL(k_trtri_cols_g, trtri_cols_body, CholInvTask, TT_NT)

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
  __shared__ double sa[GP_BK][GR_T + 2];
  __shared__ double sb[GP_BK][GR_T + 2];
  const int a0 = by * GR_T, c0 = bx * GR_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  if (q.skip && *q.skip) {                                     // pass kept: Q^T = Y^T
    for (int e = tid; e < GR_T * GR_T; e += 256) {
      const int row = a0 + e / GR_T, col = c0 + e % GR_T;
      if (row < l_pad && col < ncols) {
        const float v = (row < n) ? Yt[(long)row * ldy + col] : 0.f;
        Qt[(long)row * ldq + col] = v;
        if (Qtb) Qtb[(long)row * ldqb + col] = f32_to_bf16_rne(v);
      }
    }
    return;
  }
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
  const int kend = min(n, a0 + GR_T);
  // loaders, 32-wide K steps with the next step in registers during the MFMAs:
  //   L^{-1}: rows lr, lr + 32, k lk .. lk + 3;  Y^T: k rows kr, kr + 16, columns cc .. cc + 3
  const int lr = tid >> 3, lk = (tid & 7) * 4, kr = tid >> 4, cc = (tid & 15) * 4;
  const bool yvec = ((ldy & 3) == 0) && ((((uintptr_t)Yt) & 15) == 0);
  double ra[2][4];
  float4 rb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = a0 + lr + 32 * u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + lk + i;
        ra[u][i] = (row < n && k < kend) ? Li[(long)row * ldl + k] : 0.0;
      }
      const int k = k0 + kr + 16 * u, col = c0 + cc;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k < kend) {
        const float* y = Yt + (long)k * ldy + col;
        if (yvec && col + 4 <= ncols) {
          v = *(const float4*)y;
        } else {
          if (col + 0 < ncols) v.x = y[0];
          if (col + 1 < ncols) v.y = y[1];
          if (col + 2 < ncols) v.z = y[2];
          if (col + 3 < ncols) v.w = y[3];
        }
      }
      rb[u] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int i = 0; i < 4; ++i) sa[lk + i][lr + 32 * u] = ra[u][i];
      double* d = &sb[kr + 16 * u][cc];
      d[0] = (double)rb[u].x; d[1] = (double)rb[u].y; d[2] = (double)rb[u].z; d[3] = (double)rb[u].w;
    }
  };
  if (kend > 0) load(0);
  for (int k0 = 0; k0 < kend; k0 += GP_BK) {
    __syncthreads();                                 // the previous step's reads are done
    store();
    __syncthreads();
    if (k0 + GP_BK < kend) load(k0 + GP_BK);         // in flight during the MFMAs
#pragma unroll
    for (int kk = 0; kk < GP_BK; kk += 4) {
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
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(512), 0, s, G, ldg, n, m_rows, W, ldw, Li, status, fail_flag);
  return hipGetLastError();
}

hipError_t launch_cholinv(double* G, long ldg, int n, long m_rows, double* Linv, long ldl, int l_pad, double* dsave,
                          int* status, int* fail_flag, hipStream_t s, int* skip, double tol) {
  CholInvTask q{G, ldg, n, m_rows, Linv, ldl, l_pad, dsave, status, fail_flag, 0, skip, tol};
  hipLaunchKernelGGL(k_cholinv, dim3(1), dim3(BC_NT), 0, s, q);
  q.attempt = 1;
  hipLaunchKernelGGL(k_cholinv, dim3(1), dim3(BC_NT), 0, s, q);
  if (l_pad > BC) hipLaunchKernelGGL(k_trtri_cols, dim3(l_pad / BC - 1), dim3(TT_NT), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* Li, long ldl, int n, const float* Yt, long ldy, int ncols, float* Qt, long ldq,
                       uint16_t* Qtb, long ldqb, int l_pad, hipStream_t s, const int* skip) {
  TrmmTask q{Li, ldl, n, Yt, ldy, ncols, Qt, ldq, Qtb, ldqb, l_pad, skip};
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
KFAC_GLAUNCH(launch_cholinv_g, k_cholinv_g, CholInvTask, BC_NT)
KFAC_GLAUNCH(launch_trtri_cols_g, k_trtri_cols_g, CholInvTask, TT_NT)
int trtri_col_blocks(int l_pad) { return l_pad / BC - 1; }
KFAC_GLAUNCH(launch_trmm_g, k_trmm_f64_g, TrmmTask, 256)

int gram_reduce_slices() { return GR_T * GR_T / 256; }
int trmm_blocks_x(int ncols) { return (ncols + GR_T - 1) / GR_T; }
int trmm_blocks_y(int l_pad) { return (l_pad + GR_T - 1) / GR_T; }
}  // namespace kfac
