// fp64 kernels of the randomized eigendecomposition (Alg. 3):
//  * Gram / projection products  G = A B^T  (A, B: l x d fp32, accumulated in fp64 on
//    v_mfma_f64_16x16x4_f64, split over d with an in-order reduction);
//  * CholeskyQR: blocked right-looking Cholesky of the l x l Gram in one workgroup, with a
//    shifted retry, and the blocked forward substitution Q^T = L^{-1} Y^T;
//  * the l x l symmetric eigensolver: Householder tridiagonalisation, multisection
//    bisection on Sturm counts, inverse iteration (Gram-Schmidt inside tight clusters)
//    and the back-transformation by the Householder reflectors.
#include "kernels.h"

namespace kfac {

// ======================================================================================
// Gram / projection: C[a][b] = sum_k A[a][k] * B[b][k]   (fp32 inputs, fp64 accumulate)
// ======================================================================================
constexpr int GR_T = 64, GR_BK = 16;

struct GramP {
  const float* A; long lda;
  const float* B; long ldb;
  int L;            // rows of A and B (l_pad)
  int K;            // contraction length (d)
  int sym;          // 1: A == B, only upper tiles
  int ksplit;
  double* part;     // [tile][ks][64*64]
  double* C; long ldc;
  int* status;
};

__device__ __forceinline__ void tile_of(int t, int T, int sym, int& I, int& J) {
  if (sym) { upper_tile(t, T, I, J); }
  else { I = t / T; J = t % T; }
}

// grid (tiles, ksplit), 256 threads = 2 x 2 waves of 32 x 32.
__global__ __launch_bounds__(256) void k_gram_partial(GramP p) {
  __shared__ double sa[GR_BK][GR_T + 2];
  __shared__ double sb[GR_BK][GR_T + 2];
  const int T = (p.L + GR_T - 1) / GR_T;
  int I, J;
  tile_of(blockIdx.x, T, p.sym, I, J);
  const int a0 = I * GR_T, b0 = J * GR_T;
  const int ks = blockIdx.y, nks = gridDim.y;
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
  double* slot = p.part + ((long)blockIdx.x * nks + ks) * (GR_T * GR_T);
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

// grid (tiles): sum the K slices in order, write C (and the mirror for symmetric).
__global__ __launch_bounds__(256) void k_gram_reduce(GramP p) {
  const int T = (p.L + GR_T - 1) / GR_T;
  int I, J;
  tile_of(blockIdx.x, T, p.sym, I, J);
  const double* base = p.part + (long)blockIdx.x * p.ksplit * (GR_T * GR_T);
  bool bad = false;
  for (int e = threadIdx.x; e < GR_T * GR_T; e += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < p.ksplit; ++k) s += base[(long)k * GR_T * GR_T + e];
    int a = I * GR_T + e / GR_T, b = J * GR_T + e % GR_T;
    if (a < p.L && b < p.L) {
      if (!isfinite(s)) bad = true;
      p.C[(long)a * p.ldc + b] = s;
      if (p.sym && I != J) p.C[(long)b * p.ldc + a] = s;
    }
  }
  if (bad && p.status) atomicOr(p.status, KFAC_DS_NONFINITE);
}

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
// Forward substitution Q^T = L^{-1} Y^T, 32 columns of Y^T per workgroup (256 threads):
// for each 16-row block b:  X_b = Li_b (Y_b - sum_{c<b} L_bc X_c).  fp64 arithmetic,
// fp32 (and optional bf16) output; rows >= n are written as zero.
// ======================================================================================
constexpr int TS_NC = 32;

__global__ __launch_bounds__(256) void k_trsm(const double* W, long ldw, const double* Li, int n,
                                              int l_pad, const float* Yt, long ldy, int ncols,
                                              float* Qt, long ldq, uint16_t* Qtb, long ldqb) {
  __shared__ double X[CH_MAXN][TS_NC + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * TS_NC;
  const int nblk = (n + CH_NB - 1) / CH_NB;
  for (int e = tid; e < nblk * CH_NB * TS_NC; e += 256) {
    int i = e / TS_NC, c = e % TS_NC;
    double v = 0.0;
    if (i < n && c0 + c < ncols) v = (double)Yt[(long)i * ldy + c0 + c];
    X[i][c] = v;
  }
  __syncthreads();
  constexpr int CPT = CH_NB * TS_NC / 256;        // columns per thread
  const int il = tid / (TS_NC / CPT), cq = (tid % (TS_NC / CPT)) * CPT;
  for (int b = 0; b < nblk; ++b) {
    const int kb = b * CH_NB;
    const int i = kb + il;
    double t[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) t[u] = X[i][cq + u];
    if (i < n) {
      for (int s = 0; s < kb; ++s) {
        double l = W[(long)i * ldw + s];
#pragma unroll
        for (int u = 0; u < CPT; ++u) t[u] -= l * X[s][cq + u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CPT; ++u) X[i][cq + u] = t[u];
    __syncthreads();
    double o[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) o[u] = 0.0;
    const double* lb = Li + (long)b * CH_NB * CH_NB + il * CH_NB;
#pragma unroll
    for (int s = 0; s < CH_NB; ++s) {
      double l = lb[s];
#pragma unroll
      for (int u = 0; u < CPT; ++u) o[u] += l * X[kb + s][cq + u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < CPT; ++u) X[i][cq + u] = (i < n) ? o[u] : 0.0;
    __syncthreads();
  }
  for (int e = tid; e < l_pad * TS_NC; e += 256) {
    int i = e / TS_NC, c = e % TS_NC;
    if (c0 + c >= ncols) continue;
    float v = (i < n) ? (float)X[i][c] : 0.f;
    Qt[(long)i * ldq + c0 + c] = v;
    if (Qtb) Qtb[(long)i * ldqb + c0 + c] = f32_to_bf16_rne(v);
  }
}

// ======================================================================================
// Householder tridiagonalisation of the symmetric n x n matrix S = (C + C^T)/2
// (one workgroup, 1024 threads; working copy A in global memory, L2 resident).
// Reflector k (H_k = I - 2 v v^T, v supported on rows k+1..n-1) is stored in V row k.
// Outputs diag[n], off[n-1].  Input either fp64 C (ldc) or fp32 F (ldf) when Cf != null.
// ======================================================================================
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(1024) void k_tridiag(const double* C, long ldc, const float* Cf, long ldcf,
                                                  int n, double* A, double* V, double* diag,
                                                  double* off, int* status) {
  __shared__ double v[CH_MAXN];
  __shared__ double pw[CH_MAXN];
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool bad = false;
  for (long e = tid; e < (long)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    double a, b;
    if (Cf) { a = Cf[(long)i * ldcf + j]; b = Cf[(long)j * ldcf + i]; }
    else { a = C[(long)i * ldc + j]; b = C[(long)j * ldc + i]; }
    double s = 0.5 * (a + b);
    if (!isfinite(s)) bad = true;
    A[(long)i * n + j] = s;
  }
  if (bad) atomicOr(status, KFAC_DS_NONFINITE);
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m0 = k + 1;
    // (a) reflector from x = A[k][k+1:n]
    double part = 0.0;
    for (int j = m0 + tid; j < n; j += blockDim.x) { double x = A[(long)k * n + j]; part += x * x; }
    double nrm2 = block_sum(part, red);
    double x0 = A[(long)k * n + m0];
    double nrm = sqrt(nrm2);
    double alpha = (x0 >= 0.0) ? -nrm : nrm;
    double vn2 = nrm2 - x0 * x0 + (x0 - alpha) * (x0 - alpha);
    double inv = (nrm2 > 0.0 && vn2 > 0.0) ? 1.0 / sqrt(vn2) : 0.0;
    for (int j = tid; j < n; j += blockDim.x) {
      double x = (j > m0) ? A[(long)k * n + j] : (j == m0 ? x0 - alpha : 0.0);
      double vj = (j >= m0) ? x * inv : 0.0;
      v[j] = vj;
      V[(long)k * n + j] = vj;
    }
    if (tid == 0) { diag[k] = A[(long)k * n + k]; off[k] = (inv > 0.0) ? alpha : x0; }
    __syncthreads();
    if (inv == 0.0) continue;   // column already reduced
    // (b) p = 2 A22 v   (wave per row, lanes over columns)
    for (int i = m0 + wave; i < n; i += 16) {
      double s = 0.0;
      for (int j = m0 + lane; j < n; j += 64) s += A[(long)i * n + j] * v[j];
      s = wave_sum(s);
      if (lane == 0) pw[i] = 2.0 * s;
    }
    __syncthreads();
    // (c) w = p - (v^T p) v
    double kp = 0.0;
    for (int j = m0 + tid; j < n; j += blockDim.x) kp += v[j] * pw[j];
    double K = block_sum(kp, red);
    for (int j = m0 + tid; j < n; j += blockDim.x) pw[j] = pw[j] - K * v[j];
    __syncthreads();
    // (d) A22 -= v w^T + w v^T
    const int mm = n - m0;
    for (long e = tid; e < (long)mm * mm; e += blockDim.x) {
      int i = m0 + (int)(e / mm), j = m0 + (int)(e % mm);
      A[(long)i * n + j] -= v[i] * pw[j] + pw[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      diag[n - 2] = A[(long)(n - 2) * n + n - 2];
      off[n - 2] = A[(long)(n - 1) * n + n - 2];
    }
    diag[n - 1] = A[(long)(n - 1) * n + n - 1];
  }
}

// ======================================================================================
// Eigenpairs of the symmetric tridiagonal T = tridiag(off, diag, off) (one workgroup):
//  * eigenvalue k (k-th largest, k < r) by multisection bisection: 4 lanes per
//    eigenvalue evaluate Sturm counts (number of eigenvalues below x) at 4 interior
//    points of the bracket per step;
//  * eigenvector by inverse iteration on T - lambda I (LU with partial pivoting, three
//    solves), one thread per cluster of eigenvalues closer than ctol, with modified
//    Gram-Schmidt against the earlier members of its cluster.
// Z (n x r, fp64, row-major) receives the eigenvectors of T; D_out the eigenvalues.
// scratch: 5 * n * r doubles.
// ======================================================================================
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(1024) void k_tri_eig(const double* diag, const double* off, int n, int r,
                                                  double* Z, long ldz, double* Dout, double* scratch,
                                                  int* status) {
  __shared__ double d[CH_MAXN], e[CH_MAXN], e2[CH_MAXN];
  __shared__ double lam[CH_MAXN];
  __shared__ int cstart[CH_MAXN];
  __shared__ double sgl, sgu, spiv, stn;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) {
    d[i] = diag[i];
    double ei = (i + 1 < n) ? off[i] : 0.0;
    e[i] = ei; e2[i] = ei * ei;
  }
  __syncthreads();
  if (tid == 0) {
    double gl = d[0], gu = d[0], emax = 0.0;
    for (int i = 0; i < n; ++i) {
      double rad = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      gl = fmin(gl, d[i] - rad); gu = fmax(gu, d[i] + rad);
      if (i + 1 < n) emax = fmax(emax, e2[i]);
    }
    double tn = fmax(fabs(gl), fabs(gu));
    if (tn == 0.0) tn = 1.0;
    gl -= 2.0 * 2.2204460492503131e-16 * tn * n + 1e-300;
    gu += 2.0 * 2.2204460492503131e-16 * tn * n + 1e-300;
    sgl = gl; sgu = gu; stn = tn;
    spiv = 2.2250738585072014e-308 * fmax(1.0, emax);
  }
  __syncthreads();
  const double pivmin = spiv, tnorm = stn;
  // ---- bisection (4 lanes per eigenvalue) -------------------------------------------
  for (int base = 0; base < r; base += (int)(blockDim.x / 4)) {
    const int k = base + tid / 4, sub = tid & 3;
    const bool active = k < r;
    const int target = n - 1 - (active ? k : 0);   // ascending index of the eigenvalue
    double lo = sgl, hi = sgu;
    for (int it = 0; it < 64; ++it) {
      double w = hi - lo;
      double tol = 2.2204460492503131e-16 * (fabs(lo) + fabs(hi) + 0.01 * tnorm) + 4.0 * pivmin;
      bool done = !(w > tol);
      double x = lo + w * (double)(sub + 1) / 5.0;
      int c = (active && !done) ? sturm_count(d, e2, n, x, pivmin) : 0;
      // gather the 4 counts / points of this group
      double xs[4]; int cs[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        xs[t] = __shfl(x, (tid & ~3) + t, 64);
        cs[t] = __shfl(c, (tid & ~3) + t, 64);
      }
      bool all_done = __all(done || !active);
      if (all_done) break;
      if (!done && active) {
        double nlo = lo, nhi = hi;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (cs[t] <= target) nlo = xs[t];           // eigenvalue `target` lies above x_t
        }
#pragma unroll
        for (int t = 3; t >= 0; --t) {
          if (cs[t] >= target + 1) nhi = xs[t];
        }
        lo = nlo; hi = nhi;
      }
    }
    if (active && sub == 0) {
      double v = 0.5 * (lo + hi);
      lam[k] = v;
      Dout[k] = v;
    }
  }
  __syncthreads();
  // ---- clusters ---------------------------------------------------------------------
  const double ctol = 1e-7 * tnorm;
  for (int k = tid; k < r; k += blockDim.x) {
    cstart[k] = (k == 0 || (lam[k - 1] - lam[k]) > ctol) ? 1 : 0;
  }
  __syncthreads();
  // ---- inverse iteration: one thread per cluster -----------------------------------
  // LU of T - mu I with partial pivoting (rows i, i+1 swapped when |sub| > |diag|):
  // U has diagonal ud, superdiagonals uu, uu2; L has multipliers lf; piv marks swaps.
  // Per-thread vectors live in column k0 of [i][r] arrays (coalesced across threads);
  // every recurrence carries its running values in registers.
  const double eps = 2.2204460492503131e-16;
  double* s_lf = scratch;
  double* s_ud = scratch + (long)n * r;
  double* s_uu = scratch + 2L * n * r;
  double* s_u2 = scratch + 3L * n * r;
  double* s_pv = scratch + 4L * n * r;
  for (int k0 = tid; k0 < r; k0 += blockDim.x) {
    if (!cstart[k0]) continue;
    int kend = k0 + 1;
    while (kend < r && !cstart[kend]) ++kend;
    for (int k = k0; k < kend; ++k) {
      const double mu = lam[k] + (double)(k - k0) * 10.0 * eps * tnorm;
      double cd = d[0] - mu;                 // current (modified) diagonal of row i
      double cu = (n > 1) ? e[0] : 0.0;      // current first superdiagonal of row i
      for (int i = 0; i + 1 < n; ++i) {
        const double dl = e[i];
        const double nd = d[i + 1] - mu;
        const double nu = (i + 2 < n) ? e[i + 1] : 0.0;
        const long o = (long)i * r + k0;
        if (fabs(cd) >= fabs(dl)) {
          if (cd == 0.0) cd = eps * tnorm;
          const double f = dl / cd;
          s_lf[o] = f; s_ud[o] = cd; s_uu[o] = cu; s_u2[o] = 0.0; s_pv[o] = 0.0;
          cd = nd - f * cu;
          cu = nu;
        } else {
          const double f = cd / dl;
          s_lf[o] = f; s_ud[o] = dl; s_uu[o] = nd; s_u2[o] = nu; s_pv[o] = 1.0;
          cd = cu - f * nd;
          cu = -f * nu;
        }
      }
      if (cd == 0.0) cd = eps * tnorm;
      s_ud[(long)(n - 1) * r + k0] = cd;
      double* zc = Z + k;   // column k of Z, row stride ldz
      for (int i = 0; i < n; ++i)
        zc[(long)i * ldz] = (double)(hash32((uint32_t)(i * 7919 + k * 104729 + 17)) & 0xffffff) / 8388608.0 - 1.0;
      for (int iter = 0; iter < 3; ++iter) {
        // forward: apply the row swaps and L
        double cur = zc[0];
        for (int i = 0; i + 1 < n; ++i) {
          const long o = (long)i * r + k0;
          const double nxt = zc[(long)(i + 1) * ldz];
          const double f = s_lf[o];
          if (s_pv[o] == 0.0) { zc[(long)i * ldz] = cur; cur = nxt - f * cur; }
          else { zc[(long)i * ldz] = nxt; cur = cur - f * nxt; }
        }
        zc[(long)(n - 1) * ldz] = cur;
        // backward: U x = y
        double x1 = 0.0, x2 = 0.0;   // x_{i+1}, x_{i+2}
        for (int i = n - 1; i >= 0; --i) {
          const long o = (long)i * r + k0;
          double sv = zc[(long)i * ldz];
          if (i + 1 < n) sv -= s_uu[o] * x1;
          if (i + 2 < n) sv -= s_u2[o] * x2;
          const double xi = sv / s_ud[o];
          zc[(long)i * ldz] = xi;
          x2 = x1; x1 = xi;
        }
        // Gram-Schmidt against the earlier members of this cluster (two passes)
        for (int pass = 0; pass < 2; ++pass)
          for (int j = k0; j < k; ++j) {
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot += Z[(long)i * ldz + j] * zc[(long)i * ldz];
            for (int i = 0; i < n; ++i) zc[(long)i * ldz] -= dot * Z[(long)i * ldz + j];
          }
        double nn = 0.0;
        for (int i = 0; i < n; ++i) { const double z = zc[(long)i * ldz]; nn += z * z; }
        const double sc = (nn > 0.0 && isfinite(nn)) ? 1.0 / sqrt(nn) : 0.0;
        if (sc == 0.0) atomicOr(status, KFAC_DS_EIG_NOCONV);
        for (int i = 0; i < n; ++i) zc[(long)i * ldz] *= sc;
      }
    }
  }
}

// ======================================================================================
// Back-transformation P = H_0 H_1 ... H_{n-3} Z for the first r columns, one wavefront
// per column, reflectors applied from the last to the first.  Output fp32 P (ldp) with
// rows n..n_pad-1 zero.  grid = ceil(r/4) blocks of 256 threads.
// ======================================================================================
__global__ __launch_bounds__(256) void k_backtransform(const double* V, const double* Z, long ldz,
                                                       int n, int n_pad, int r, float* P, long ldp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave;
  if (c >= r) return;
  constexpr int PER = CH_MAXN / 64;
  double z[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    int i = lane + 64 * u;
    z[u] = (i < n) ? Z[(long)i * ldz + c] : 0.0;
  }
  for (int k = n - 3; k >= 0; --k) {
    const double* vk = V + (long)k * n;
    double vv[PER];
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      int i = lane + 64 * u;
      vv[u] = (i > k && i < n) ? vk[i] : 0.0;
      s += vv[u] * z[u];
    }
    s = 2.0 * wave_sum(s);
#pragma unroll
    for (int u = 0; u < PER; ++u) z[u] -= s * vv[u];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    int i = lane + 64 * u;
    if (i < n_pad) P[(long)i * ldp + c] = (i < n) ? (float)z[u] : 0.f;
  }
}

__global__ void k_d64_to_f32(const double* a, float* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

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

hipError_t launch_gram(const float* A, long lda, const float* B, long ldb, int L, int K, int sym,
                       double* part, double* C, long ldc, int* status, hipStream_t s) {
  GramP p{A, lda, B, ldb, L, K, sym, gram_ksplit(L, K, sym), part, C, ldc, status};
  int T = (L + GR_T - 1) / GR_T;
  int tiles = sym ? T * (T + 1) / 2 : T * T;
  hipLaunchKernelGGL(k_gram_partial, dim3(tiles, p.ksplit), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_gram_reduce, dim3(tiles), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* G, long ldg, int n, long m_rows, double* W, long ldw,
                           double* Li, int* status, int* fail_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(512), 0, s, G, ldg, n, m_rows, W, ldw, Li, status, fail_flag);
  return hipGetLastError();
}

hipError_t launch_trsm(const double* W, long ldw, const double* Li, int n, int l_pad, const float* Yt,
                       long ldy, int ncols, float* Qt, long ldq, uint16_t* Qtb, long ldqb, hipStream_t s) {
  hipLaunchKernelGGL(k_trsm, dim3((ncols + TS_NC - 1) / TS_NC), dim3(256), 0, s, W, ldw, Li, n, l_pad, Yt,
                     ldy, ncols, Qt, ldq, Qtb, ldqb);
  return hipGetLastError();
}

hipError_t launch_small_eig(const double* C, long ldc, const float* Cf, long ldcf, int n, int n_pad, int r,
                            double* A, double* V, double* diag, double* off, double* Z, double* scratch,
                            float* P, long ldp, float* D, double* Dd, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(1024), 0, s, C, ldc, Cf, ldcf, n, A, V, diag, off, status);
  hipLaunchKernelGGL(k_tri_eig, dim3(1), dim3(1024), 0, s, diag, off, n, r, Z, (long)r, Dd, scratch, status);
  hipLaunchKernelGGL(k_backtransform, dim3((r + 3) / 4), dim3(256), 0, s, V, Z, (long)r, n, n_pad, r, P, ldp);
  hipLaunchKernelGGL(k_d64_to_f32, dim3((r + 255) / 256), dim3(256), 0, s, Dd, D, r);
  return hipGetLastError();
}

}  // namespace kfac
