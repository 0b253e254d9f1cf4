// fp64 symmetric eigensolver for the (r+p) x (r+p) Rayleigh-Ritz matrix of Alg. 3
// ("Eigen_decomp(C)"), and for the factor itself when r+p >= d:
//   1. Householder tridiagonalisation, one workgroup.  For n <= 288 the lower triangle
//      lives in registers of 512 threads (16 x 32 thread grid, two rows per thread in
//      each of the 9 x 9 blocks of 32) and the diagonal blocks in LDS.
//   2. split of the tridiagonal T into unreduced blocks (|e_i| <= 2 eps ||T||);
//   3. every eigenvalue of every block by 16-way multisection bisection on Sturm counts
//      (one 16-lane group per eigenvalue, many workgroups);
//   4. selection of the r largest (descending), detection of tight clusters;
//   5. eigenvectors by the twisted factorisation T - lambda I = N_k Delta_k N_k^T of the
//      eigenvalue's block (one thread per eigenvector, factors kept in LDS);
//   6. inverse iteration with Gram-Schmidt for members of tight clusters (rare);
//   7. back-transformation by the Householder reflectors (eight lanes per column).
#include <utility>
#include "kernels.h"

namespace kfac {

constexpr double kEps = 2.2204460492503131e-16;
constexpr double kTiny = 2.2250738585072014e-308;

// ======================================================================================
// 1a. Tridiagonalisation for n <= 288 with the matrix held on chip, 512 threads.
// Thread t: tr = t / 32 (0..15), tc = t % 32 owns A[32 I + tr + 16 h][32 J + tc], h = 0, 1,
// of the lower triangle: the 36 off-diagonal blocks (I > J) in registers (slot
// I (I - 1) / 2 + J), the 9 diagonal blocks in LDS in full (Ld[I][row][col], both
// triangles, each updated by the same rank-2 formula; the lower one is read out).  Block
// columns are processed by a template per block column so every register index is a
// constant.  One Householder step costs three barriers:
//   column k (rows > k) is in scol[k & 1]; every wave derives the reflector from it
//   (same data, same reduction order, so the same bits in every wave) -> p = 2 A v,
//   row sums reduced in the wave, column partials per wave -> barrier -> p reduced ->
//   barrier -> K = v^T p (every wave), w = p - K v on the fly, rank-2 update, the owners
//   of column k + 1 copy it into the other buffer -> barrier.
// ======================================================================================
constexpr int TB = 32, TNB = 9, TNMAX = TB * TNB, TNT = 512, TNW = TNT / 64;
// thread rows of the 32 x 32 block grid and rows per thread in each block
constexpr int TTR = TNT / TB, THR = TB / TTR;

__device__ __forceinline__ constexpr int toff(int I, int J) { return I * (I - 1) / 2 + J; }   // I > J

struct TriSh {
  double (*Ld)[TB][TB + 1];
  double (*scol)[TNMAX];    // two column buffers
  double* sv;               // v of the current step (written by every wave, same values)
  double* sp;               // p = 2 A v, zero on rows <= k
  double (*spr)[TB][8];     // row partials, one per 4 columns of a block
  double (*spc)[TNB][TB];   // column partials per wave
};

// Column kn of the working matrix (rows >= kn) into dst by its owners (tc == kn % 32, block
// column JN): entries they hold themselves, already updated, so no barrier is needed first.
template <int JN>
__device__ __forceinline__ void tri_copy_col(const double (&a)[36][THR], const TriSh& S, int n, int kn, double* dst) {
  if constexpr (JN < TNB) {
    const int t = threadIdx.x, tr = t >> 5, tc = t & 31;
    if (tc != (kn & 31)) return;
#pragma unroll
    for (int h = 0; h < THR; ++h) {
      const int rr = tr + TTR * h;
      {
        const int i = TB * JN + rr;
        if (rr >= tc && i < n) dst[i] = S.Ld[JN][rr][tc];
      }
#pragma unroll
      for (int I = JN + 1; I < TNB; ++I) {
        const int i = TB * I + rr;
        if (i < n) dst[i] = a[toff(I, JN)][h];
      }
    }
  }
}

// Step k = 32 J0 + c0; LASTC: c0 is the block column's last (then the trailing blocks
// start at J0 + 1, else at J0; a template parameter, so every block predicate below is a
// compile-time constant).
template <int J0, bool LASTC>
__device__ __forceinline__ void tri_step(double (&a)[36][THR], const TriSh& S, int n, double* V, double* diag,
                                         double* off, int c0) {
  const int t = threadIdx.x, tr = t >> 5, tc = t & 31, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  double (*Ld)[TB][TB + 1] = S.Ld;
  {
    const int k = TB * J0 + c0;
    constexpr int kb = J0 + (LASTC ? 1 : 0);          // first block with rows/cols > k
    const double* col = S.scol[k & 1];
    // (1) reflector H = I - 2 v v^T (|v| = 1) from column k, in every wave.  The lane's
    // entries of the column (i = lane + 64 u) are read once, all loads issued together.
    constexpr int TCU = (TNMAX + 63) / 64;
    double cx[TCU];
#pragma unroll
    for (int u = 0; u < TCU; ++u) {
      const int i = lane + 64 * u;
      cx[u] = (i < TNMAX) ? col[i] : 0.0;
    }
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < TCU; ++u) {
      const int i = lane + 64 * u;
      if (i > k && i < n) s2 += cx[u] * cx[u];
    }
    s2 = wave_sum(s2);
    const double x0 = col[k + 1];
    // |x|, alpha = -sign(x0) |x| and 1 / |x - alpha e1| with |x - alpha e1|^2 =
    // 2 |x| (|x| + |x0|), by Newton-refined reciprocal square roots (short dependency chain)
    const double nrm = (s2 > 0.0) ? s2 * rsqrt_nr(s2) : 0.0;
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double vn2 = 2.0 * nrm * (nrm + fabs(x0));
    const double inv = (s2 > 0.0 && vn2 > 0.0) ? rsqrt_nr(vn2) : 0.0;
    const double v1 = (x0 - alpha) * inv;
    // v into LDS by every wave (identical values; the wave's own stores precede its
    // loads in LDS order, and the previous step's readers are past the last barrier)
#pragma unroll
    for (int u = 0; u < TCU; ++u) {
      const int i = lane + 64 * u;
      if (i < TNMAX) {
        const double vi = (i > k + 1 && i < n) ? cx[u] * inv : (i == k + 1 ? v1 : 0.0);
        S.sv[i] = vi;
        if (wave == 0 && i < n) V[(long)k * n + i] = vi;
      }
    }
    if (wave == 0 && lane == 0) {
      diag[k] = col[k];
      off[k] = (inv > 0.0) ? alpha : x0;
    }
    auto vval = [&](int i) { return S.sv[i]; };
    if (inv != 0.0) {                                 // uniform: same value in every wave
      // (2) p = 2 A v: v at the thread's columns once, at its rows once per block row
      double vc[TNB], pc[TNB];
#pragma unroll
      for (int J = J0; J < TNB; ++J) { vc[J] = (J >= kb) ? vval(TB * J + tc) : 0.0; pc[J] = 0.0; }
#pragma unroll
      for (int I = J0; I < TNB; ++I) {
        if (I >= kb) {
#pragma unroll
          for (int h = 0; h < THR; ++h) {
            const int rr = tr + TTR * h;
            const double vi = vval(TB * I + rr);
            double pr = 0.0;
#pragma unroll
            for (int J = J0; J < I; ++J) {
              if (J >= kb) {
                const double aij = a[toff(I, J)][h];
                pr += aij * vc[J];
                pc[J] += aij * vi;
              }
            }
            pr += Ld[I][rr][tc] * vc[I];             // diagonal block I, held in full
            pr += dpp_any<0xB1>(pr);                 // sum over 4 neighbouring columns
            pr += dpp_any<0x4E>(pr);
            S.spr[I][rr][tc >> 2] = pr;              // the 4 lanes store the same value
          }
        }
      }
#pragma unroll
      for (int J = J0; J < TNB; ++J) {
        if (J >= kb) {
          const double y = pc[J] + __shfl_xor(pc[J], 32, 64);
          if (lane < 32) S.spc[wave][J][tc] = y;
        }
      }
      __syncthreads();
      if (t < TNMAX) {
        double p = 0.0;
        if (t > k && t < n) {
          const int I = t >> 5, c = t & 31;
          p = ((S.spr[I][c][0] + S.spr[I][c][1]) + (S.spr[I][c][2] + S.spr[I][c][3])) +
              ((S.spr[I][c][4] + S.spr[I][c][5]) + (S.spr[I][c][6] + S.spr[I][c][7]));
#pragma unroll
          for (int w2 = 0; w2 < TNW; ++w2) p += S.spc[w2][I][c];
        }
        S.sp[t] = 2.0 * p;
      }
      __syncthreads();
      // (3) K = v^T p in every wave; w = p - K v (zero on rows <= k); A -= v w^T + w v^T
      double kp = 0.0;
#pragma unroll
      for (int u = 0; u < TCU; ++u) {
        const int i = lane + 64 * u;
        if (i > k && i < n) kp += vval(i) * S.sp[i];
      }
      const double K = wave_sum(kp);
      double wc[TNB];
#pragma unroll
      for (int J = J0; J < TNB; ++J) wc[J] = (J >= kb) ? S.sp[TB * J + tc] - K * vc[J] : 0.0;
#pragma unroll
      for (int I = J0; I < TNB; ++I) {
        if (I >= kb) {
#pragma unroll
          for (int h = 0; h < THR; ++h) {
            const int rr = tr + TTR * h;
            const double vi = vval(TB * I + rr), wi = S.sp[TB * I + rr] - K * vi;
#pragma unroll
            for (int J = J0; J < I; ++J)
              if (J >= kb) a[toff(I, J)][h] = fma(-wi, vc[J], fma(-vi, wc[J], a[toff(I, J)][h]));
            Ld[I][rr][tc] = fma(-wi, vc[I], fma(-vi, wc[I], Ld[I][rr][tc]));
          }
        }
      }
    }
    // (4) column k + 1 into the other buffer (its owners updated it just now)
    tri_copy_col<J0 + (LASTC ? 1 : 0)>(a, S, n, k + 1, S.scol[(k + 1) & 1]);
    __syncthreads();
  }
}

template <int J0>
__device__ __forceinline__ void tri_block_col(double (&a)[36][THR], const TriSh& S, int n, double* V, double* diag,
                                              double* off) {
  if (TB * J0 + 2 >= n) return;                       // uniform
  for (int c0 = 0; c0 < TB - 1; ++c0) {
    if (TB * J0 + c0 + 2 >= n) return;                // uniform
    tri_step<J0, false>(a, S, n, V, diag, off, c0);
  }
  if (TB * J0 + TB - 1 + 2 >= n) return;
  tri_step<J0, true>(a, S, n, V, diag, off, TB - 1);
}

template <int... Js>
__device__ __forceinline__ void tri_all_cols(std::integer_sequence<int, Js...>, double (&a)[36][THR], const TriSh& S,
                                             int n, double* V, double* diag, double* off) {
  (tri_block_col<Js>(a, S, n, V, diag, off), ...);
}

__device__ __forceinline__ void tridiag_reg_body(const EigTask& q, int, int) {
  const double* C = q.C; const long ldc = q.ldc; const float* Cf = q.Cf; const long ldcf = q.ldcf;
  const int n = q.n; double* V = q.V; double* diag = q.diag; double* off = q.off; int* status = q.status;
  __shared__ double Ld[TNB][TB][TB + 1];
  __shared__ double scol[2][TNMAX];
  __shared__ double sv[TNMAX];
  __shared__ double sp[TNMAX];
  __shared__ double spr[TNB][TB][8];
  __shared__ double spc[TNW][TNB][TB];
  const int t = threadIdx.x, tr = t >> 5, tc = t & 31;
  double a[36][THR];
  bool bad = false;
  auto sym = [&](int i, int j) -> double {
    double x, y;
    if (Cf) { x = Cf[(long)i * ldcf + j]; y = Cf[(long)j * ldcf + i]; }
    else { x = C[(long)i * ldc + j]; y = C[(long)j * ldc + i]; }
    const double v = 0.5 * (x + y);
    if (!isfinite(v)) bad = true;
    return v;
  };
#pragma unroll
  for (int I = 0; I < TNB; ++I) {
#pragma unroll
    for (int h = 0; h < THR; ++h) {
      const int rr = tr + TTR * h, i = TB * I + rr;
      {
        const int j = TB * I + tc;
        Ld[I][rr][tc] = (i < n && j < n) ? sym(i, j) : 0.0;
      }
#pragma unroll
      for (int J = 0; J < I; ++J) {
        const int j = TB * J + tc;
        a[toff(I, J)][h] = (i < n && j < n) ? sym(i, j) : 0.0;
      }
    }
  }
  if (bad) atomicOr(status, KFAC_DS_NONFINITE);
  for (int i = t; i < TNMAX; i += TNT) { scol[0][i] = 0.0; scol[1][i] = 0.0; sv[i] = 0.0; sp[i] = 0.0; }
  __syncthreads();
  TriSh S{Ld, scol, sv, sp, spr, spc};
  tri_copy_col<0>(a, S, n, 0, scol[0]);
  __syncthreads();
  tri_all_cols(std::make_integer_sequence<int, TNB>{}, a, S, n, V, diag, off);
  // trailing 2 x 2 (or 1 x 1) block
  __syncthreads();
  if (t == 0) {
    if (n >= 2) diag[n - 2] = Ld[(n - 2) >> 5][(n - 2) & 31][(n - 2) & 31];
    diag[n - 1] = Ld[(n - 1) >> 5][(n - 1) & 31][(n - 1) & 31];
  }
  if (n >= 2) {
    const int i = n - 1, j = n - 2;
    if ((i >> 5) == (j >> 5)) {
      if (t == 0) off[n - 2] = Ld[i >> 5][i & 31][j & 31];
    } else {
      // (n-1, n-2) lies in the off-diagonal block (I, I-1): owner row i & 31, column j & 31
#pragma unroll
      for (int I = 1; I < TNB; ++I)
#pragma unroll
        for (int h = 0; h < THR; ++h)
          if (I == (i >> 5) && tr + TTR * h == (i & 31) && tc == (j & 31)) off[n - 2] = a[toff(I, I - 1)][h];
    }
  }
}

// ======================================================================================
// 1b. Tridiagonalisation for 288 < n <= 512: working copy in global memory (L2 resident).
// ======================================================================================
__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(1024) void k_tridiag_gmem(EigTask q) {
  const double* C = q.C; const long ldc = q.ldc; const float* Cf = q.Cf; const long ldcf = q.ldcf;
  const int n = q.n; double* A = q.A; double* V = q.V; double* diag = q.diag; double* off = q.off;
  int* status = q.status;
  __shared__ double v[KFAC_MAX_SKETCH];
  __shared__ double pw[KFAC_MAX_SKETCH];
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool bad = false;
  for (long e = tid; e < (long)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    double x, y;
    if (Cf) { x = Cf[(long)i * ldcf + j]; y = Cf[(long)j * ldcf + i]; }
    else { x = C[(long)i * ldc + j]; y = C[(long)j * ldc + i]; }
    double s = 0.5 * (x + y);
    if (!isfinite(s)) bad = true;
    A[(long)i * n + j] = s;
  }
  if (bad) atomicOr(status, KFAC_DS_NONFINITE);
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m0 = k + 1;
    double part = 0.0;
    for (int j = m0 + tid; j < n; j += blockDim.x) { double x = A[(long)k * n + j]; part += x * x; }
    double nrm2 = block_sum_1024(part, red);
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
    if (inv == 0.0) continue;
    for (int i = m0 + wave; i < n; i += 16) {
      double s = 0.0;
      for (int j = m0 + lane; j < n; j += 64) s += A[(long)i * n + j] * v[j];
      s = wave_sum(s);
      if (lane == 0) pw[i] = 2.0 * s;
    }
    __syncthreads();
    double kp = 0.0;
    for (int j = m0 + tid; j < n; j += blockDim.x) kp += v[j] * pw[j];
    double K = block_sum_1024(kp, red);
    for (int j = m0 + tid; j < n; j += blockDim.x) pw[j] = pw[j] - K * v[j];
    __syncthreads();
    const int mm = n - m0;
    for (long e = tid; e < (long)mm * mm; e += blockDim.x) {
      int i = m0 + (int)(e / mm), j = m0 + (int)(e % mm);
      A[(long)i * n + j] -= v[i] * pw[j] + pw[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) { diag[n - 2] = A[(long)(n - 2) * n + n - 2]; off[n - 2] = A[(long)(n - 1) * n + n - 2]; }
    diag[n - 1] = A[(long)(n - 1) * n + n - 1];
  }
}

// ======================================================================================
// 2. Split into unreduced blocks.  meta layout: see TriMeta.
// ======================================================================================
__device__ __forceinline__ void tri_prep_body(const EigTask& q, int, int) {
  const double* diag = q.diag; const double* off = q.off; const int n = q.n; const TriMeta& m = q.m;
  __shared__ double sred[8];
  __shared__ double ssh[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double g = 0.0, e2max = 0.0;
  for (int i = tid; i < n; i += blockDim.x) {
    double rad = (i > 0 ? fabs(off[i - 1]) : 0.0) + (i + 1 < n ? fabs(off[i]) : 0.0);
    g = fmax(g, fabs(diag[i]) + rad);
    if (i + 1 < n) e2max = fmax(e2max, off[i] * off[i]);
  }
  for (int o = 32; o >= 1; o >>= 1) { g = fmax(g, __shfl_xor(g, o, 64)); e2max = fmax(e2max, __shfl_xor(e2max, o, 64)); }
  if (lane == 0) sred[wave] = g;
  __syncthreads();
  if (tid == 0) {
    double tn = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tn = fmax(tn, sred[w]);
    if (tn == 0.0) tn = 1.0;
    ssh[0] = tn;
  }
  __syncthreads();
  if (lane == 0) sred[wave] = e2max;
  __syncthreads();
  if (tid == 0) {
    double em = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) em = fmax(em, sred[w]);
    ssh[1] = kTiny * fmax(1.0, em);
    m.scal[0] = ssh[0];
    m.scal[1] = ssh[1];
    m.scal[2] = 0.0;
  }
  __syncthreads();
  const double tn = ssh[0];
  // unreduced blocks: row i ends a block when i = n - 1 or its (negligible) off-diagonal
  // was set to zero.  The end flags go into 64-bit words (one ballot per wavefront), and
  // every row finds the nearest ends below and at or above it a word at a time.
  __shared__ unsigned long long wend[(KFAC_MAX_SKETCH + 63) / 64];
  for (int i0 = 0; i0 < n; i0 += blockDim.x) {               // uniform: ballots
    const int i = i0 + tid;
    bool f = false;
    if (i < n) {
      double e = (i + 1 < n) ? off[i] : 0.0;
      if (fabs(e) <= 2.0 * kEps * tn) e = 0.0;
      m.es[i] = e;
      f = (i == n - 1 || e == 0.0);
    }
    const unsigned long long b = __ballot(f);
    if (lane == 0 && i0 + 64 * wave < n) wend[(i0 >> 6) + wave] = b;
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    int w = i >> 6;
    unsigned long long mk = wend[w] & ((1ull << (i & 63)) - 1);   // ends before row i
    while (mk == 0 && w > 0) mk = wend[--w];
    const int lo = mk ? 64 * w + 64 - __clzll(mk) : 0;
    w = i >> 6;
    mk = wend[w] & ~((1ull << (i & 63)) - 1);                     // ends at or after row i
    while (mk == 0) mk = wend[++w];                               // row n - 1 ends the last
    m.blo[i] = lo;
    m.bhi[i] = 64 * w + __ffsll((long long)mk);
  }
}

// ======================================================================================
// 3. Bisection.  Task j (one per row) = eigenvalue number j - blo[j] (ascending) of its
// block; 16 lanes evaluate the Sturm count at 16 interior points of the bracket (each step
// narrows it 17-fold).  The counts are monotone in the point, so one ballot locates the new
// bracket.  (64 points per task, nine steps instead of thirteen, measured slower: the
// launch is bound by the fp64 work of the recurrences, which grows with the points.)
// ======================================================================================
// a / b from the hardware reciprocal (about 2^-26 relative) and one Newton step (relative
// error then about 2^-52 plus rounding): a Sturm count only needs each pivot to a few ulps,
// which perturbs the tridiagonal matrix by as much (backward stable recurrence)
__device__ __forceinline__ double fast_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = r * fma(-b, r, 2.0);
  return a * r;
}

__device__ int sturm_block(const double* d, const double* e2, int lo, int hi, double x, double pivmin) {
  int cnt = 0;
  double q = d[lo] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
#pragma unroll 4
  for (int i = lo + 1; i < hi; ++i) {
    q = (d[i] - x) - fast_div(e2[i - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

constexpr int BIS_LANES = 16;
constexpr int BIS_PER_BLOCK = 256 / BIS_LANES;

__device__ __forceinline__ void tri_bisect_body(const EigTask& q, int bx, int) {
  const double* diag = q.diag; const int n = q.n; const TriMeta& m = q.m;
  __shared__ double d[KFAC_MAX_SKETCH], e2[KFAC_MAX_SKETCH], ea[KFAC_MAX_SKETCH];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += blockDim.x) {
    d[i] = diag[i];
    double e = m.es[i];
    e2[i] = e * e;
    ea[i] = fabs(e);
  }
  __syncthreads();
  const double tn = m.scal[0], pivmin = m.scal[1];
  const int j = bx * BIS_PER_BLOCK + tid / BIS_LANES;
  const int sub = tid % BIS_LANES;
  const bool active = j < n;
  const int jj = active ? j : 0;
  const int lo_i = m.blo[jj], hi_i = m.bhi[jj];
  const int target = jj - lo_i;
  double lo = 1e300, hi = -1e300;
  for (int i = lo_i; i < hi_i; ++i) {
    double rad = (i > lo_i ? ea[i - 1] : 0.0) + (i + 1 < hi_i ? ea[i] : 0.0);
    lo = fmin(lo, d[i] - rad);
    hi = fmax(hi, d[i] + rad);
  }
  const double pad = 4.0 * kEps * tn * (hi_i - lo_i) + 2.0 * pivmin;
  lo -= pad; hi += pad;
  const int base = (threadIdx.x & 63) & ~(BIS_LANES - 1);
  // point p of the bracket; the bracket update evaluates the same expression
  auto point = [&](double l, double wd, int p) { return l + wd * (double)(p + 1) / (double)(BIS_LANES + 1); };
  for (int it = 0; it < 40; ++it) {
    const double w = hi - lo;
    const bool done = !(w > 2.0 * kEps * (fabs(lo) + fabs(hi)) + 1e-3 * kEps * tn + 4.0 * pivmin);
    const double x = point(lo, w, sub);
    const int c = (active && !done) ? sturm_block(d, e2, lo_i, hi_i, x, pivmin) : 0;
    // the counts grow with the point: the number P of points with count <= target (one
    // ballot) gives the new bracket [point P - 1, point P]
    const unsigned long long bl = __ballot(c <= target);
    constexpr unsigned long long lanes_mask = BIS_LANES == 64 ? ~0ull : ((1ull << (BIS_LANES & 63)) - 1);
    const int P = __popcll((bl >> base) & lanes_mask);
    const double nlo = (P > 0) ? point(lo, w, P - 1) : lo;
    const double nhi = (P < BIS_LANES) ? point(lo, w, P) : hi;
    if (__all(done || !active)) break;
    if (!done) { lo = nlo; hi = nhi; }
  }
  if (active && sub == 0) m.lam[j] = 0.5 * (lo + hi);
}

// ======================================================================================
// 4. Descending selection of the r largest eigenvalues and tight-cluster flags.
// ======================================================================================
__device__ __forceinline__ void tri_select_body(const EigTask& q, int, int) {
  const int n = q.n, r = q.r; const TriMeta& m = q.m; double* Dd = q.Dd; float* D = q.D;
  __shared__ double lam[KFAC_MAX_SKETCH];
  const int tid = threadIdx.x;
  // the order key maps NaN (a non-finite factor) to -inf, so that the ranks stay a
  // permutation of 0..n-1 and every col_task entry below r is written with a valid row
  for (int i = tid; i < n; i += blockDim.x) lam[i] = isnan(m.lam[i]) ? -INFINITY : m.lam[i];
  __syncthreads();
  for (int j = tid; j < n; j += blockDim.x) {
    const double lj = lam[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double li = lam[i];
      rank += (li > lj) || (li == lj && i < j);
    }
    if (rank < r) {
      const double v = m.lam[j];
      m.col_task[rank] = j;
      Dd[rank] = v;
      D[rank] = q.svd ? (float)sqrt(fmax(v, 0.0)) : (float)v;
    }
  }
  __threadfence_block();
  __syncthreads();
  // Twisted-factorisation vectors of eigenvalues a gap g apart lose orthogonality of about
  // 2 eps ||T|| / g; below g = 1e-9 ||T|| (loss above ~5e-7) members take the cluster pass.
  const double ctol = 1e-9 * m.scal[0];
  int any = 0;
  for (int k = tid; k < r; k += blockDim.x) {
    int s = 1;
    if (k > 0) {
      const int a = m.col_task[k - 1], b = m.col_task[k];
      if (m.blo[a] == m.blo[b] && fabs(lam[a] - lam[b]) <= ctol) s = 0;
    }
    m.cstart[k] = s;
    any |= (s == 0);
  }
  if (any) m.scal[2] = 1.0;   // benign race: every writer stores the same value
}

// ======================================================================================
// 5. Eigenvectors by twisted factorisation (one thread per output column).
// Forward  T - lam I = L D+ L^T :  D+_0 = d_0 - lam,  L_i = e_i / D+_i,
//                                  D+_{i+1} = d_{i+1} - lam - L_i e_i;
// backward T - lam I = U D- U^T :  D-_{m-1} = d_{m-1} - lam,  U_i = e_i / D-_{i+1},
//                                  D-_i = d_i - lam - U_i e_i;
// twist gamma_k = D+_k + D-_k - (d_k - lam), k* = argmin |gamma_k|;
// z_{k*} = 1, z_i = -L_i z_{i+1} (i < k*), z_{i+1} = -U_i z_i (i >= k*).
// The column is written unnormalised (the back-transformation normalises it).
// ======================================================================================
template <int NT, int NMAX>
__device__ __forceinline__ void tri_vec_body(const EigTask& q, int bx, int) {
  const int n = q.n, r = q.r; const TriMeta& m = q.m; double* Z = q.Z;
  const long ldz = q.ldz;
  // thread t's entry i at [i][t]: the threads of one step touch consecutive words (one
  // row per thread would put all of them in one LDS bank)
  __shared__ double sL[NMAX][NT];
  __shared__ double sD[NMAX][NT];
  // T's diagonal and off-diagonal in LDS: the recurrences read them at LDS latency
  __shared__ double td[NMAX], te[NMAX];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += NT) {
    td[i] = q.diag[i];
    te[i] = m.es[i];
  }
  __syncthreads();
  const int k = bx * NT + tid;
  if (k >= r) return;
  const double pivmin = m.scal[1];
  const double tiny = fmax(pivmin, kEps * kEps * m.scal[0]);
  const int j = m.col_task[k];
  const double lam = m.lam[j];
  const int b0 = m.blo[j], b1 = m.bhi[j];
  auto L = [&](int i) -> double& { return sL[i][tid]; };
  auto Dp = [&](int i) -> double& { return sD[i][tid]; };
  // forward
  // divisions by the pivots: hardware reciprocal + one Newton step (about 2^-52 relative,
  // a rounding-sized perturbation of each pivot); loops unrolled so that the reads of d
  // and e go out ahead of the dependent recurrence
  double dp = td[b0] - lam;
#pragma unroll 4
  for (int i = b0; i + 1 < b1; ++i) {
    if (fabs(dp) < tiny) dp = (dp < 0.0) ? -tiny : tiny;
    const double e = te[i];
    const double l = fast_div(e, dp);
    L(i - b0) = l;
    Dp(i - b0) = dp;
    dp = (td[i + 1] - lam) - l * e;
  }
  Dp(b1 - 1 - b0) = dp;
  // backward with twist search
  double dm = td[b1 - 1] - lam;
  double best = fabs(dp);   // gamma_{b1-1} = D+_{b1-1}
  int kstar = b1 - 1;
#pragma unroll 4
  for (int i = b1 - 2; i >= b0; --i) {
    if (fabs(dm) < tiny) dm = (dm < 0.0) ? -tiny : tiny;
    const double e = te[i];
    const double u = fast_div(e, dm);
    const double dmi = (td[i] - lam) - u * e;
    const double g = Dp(i - b0) + dmi - (td[i] - lam);
    Dp(i - b0) = u;           // slot i now holds U_i
    if (fabs(g) < best) { best = fabs(g); kstar = i; }
    dm = dmi;
  }
  // assemble
  for (int i = 0; i < b0; ++i) Z[(long)i * ldz + k] = 0.0;
  for (int i = b1; i < n; ++i) Z[(long)i * ldz + k] = 0.0;
  double z = 1.0;
  Z[(long)kstar * ldz + k] = 1.0;
#pragma unroll 4
  for (int i = kstar - 1; i >= b0; --i) {
    z = -L(i - b0) * z;
    Z[(long)i * ldz + k] = z;
  }
  z = 1.0;
#pragma unroll 4
  for (int i = kstar; i + 1 < b1; ++i) {
    z = -Dp(i - b0) * z;
    Z[(long)(i + 1) * ldz + k] = z;
  }
}

// ======================================================================================
// 6. Tight clusters: inverse iteration on the block with Gram-Schmidt against the earlier
// members (sequential over members, one workgroup).  Exits at once if there is none.
// The block's tridiagonal, its LU factors and the iterate live in LDS: the two serial
// sweeps (one thread) touch only LDS, the rest is spread over the workgroup.  Each
// Gram-Schmidt pass is classical (all projections of one pass computed together: one
// wavefront per earlier column, then one row-wise update), two passes per solve, so a
// member costs a fixed number of barriers however many members precede it.
// ======================================================================================
__device__ __forceinline__ void tri_cluster_body(const EigTask& q, int, int) {
  const double* diag = q.diag; const int r = q.r; const TriMeta& m = q.m; double* Z = q.Z;
  const long ldz = q.ldz; int* status = q.status;
  __shared__ double red[16];
  __shared__ double sdot;
  __shared__ double sd[KFAC_MAX_SKETCH], se[KFAC_MAX_SKETCH];        // block of T
  __shared__ double lf[KFAC_MAX_SKETCH], rud[KFAC_MAX_SKETCH];       // multipliers, 1 / U diagonal
  __shared__ double uu[KFAC_MAX_SKETCH], u2[KFAC_MAX_SKETCH];        // U super-diagonals
  __shared__ double zc[KFAC_MAX_SKETCH];                              // the iterate
  __shared__ unsigned char pv[KFAC_MAX_SKETCH];                        // row interchange at i
  __shared__ double dots[KFAC_MAX_SKETCH];                            // projections of one pass
  if (m.scal[2] == 0.0) return;
  const int tid = threadIdx.x, nw = blockDim.x >> 6;
  const double tn = m.scal[0];
  auto block_sum = [&](double v) -> double {
    v = wave_sum(v);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w];
      sdot = t;
    }
    __syncthreads();
    const double t = sdot;
    __syncthreads();                                   // red / sdot reusable
    return t;
  };
  for (int k = 1; k < r; ++k) {
    if (m.cstart[k]) continue;
    int k0 = k;
    while (k0 > 0 && !m.cstart[k0]) --k0;
    const int j = m.col_task[k];
    const int b0 = m.blo[j], b1 = m.bhi[j], nb = b1 - b0;
    const double mu = m.lam[j] + (double)(k - k0) * 10.0 * kEps * tn;
    for (int i = tid; i < nb; i += blockDim.x) {
      sd[i] = diag[b0 + i] - mu;
      se[i] = (i + 1 < nb) ? m.es[b0 + i] : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      // LU with partial pivoting of the block of T - mu I (U diagonal kept in rud)
      double cd = sd[0], cu = (nb > 1) ? se[0] : 0.0;
      for (int i = 0; i + 1 < nb; ++i) {
        const double dl = se[i], nd = sd[i + 1], nu = (i + 2 < nb) ? se[i + 1] : 0.0;
        if (fabs(cd) >= fabs(dl)) {
          if (cd == 0.0) cd = kEps * tn;
          const double f = dl / cd;
          lf[i] = f; rud[i] = cd; uu[i] = cu; u2[i] = 0.0; pv[i] = 0;
          cd = nd - f * cu; cu = nu;
        } else {
          const double f = cd / dl;
          lf[i] = f; rud[i] = dl; uu[i] = nd; u2[i] = nu; pv[i] = 1;
          cd = cu - f * nd; cu = -f * nu;
        }
      }
      rud[nb - 1] = (cd == 0.0) ? kEps * tn : cd;
      uu[nb - 1] = 0.0;
      u2[nb - 1] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < nb; i += blockDim.x) rud[i] = 1.0 / rud[i];
    for (int i = tid; i < nb; i += blockDim.x) zc[i] = Z[(long)(b0 + i) * ldz + k];
    __syncthreads();
    for (int iter = 0; iter < 3; ++iter) {
      if (tid == 0) {
        // forward: apply the interchanges and multipliers; backward: solve with U
        double cur = zc[0];
        for (int i = 0; i + 1 < nb; ++i) {
          const double nxt = zc[i + 1];
          if (pv[i] == 0) { zc[i] = cur; cur = nxt - lf[i] * cur; }
          else { zc[i] = nxt; cur = cur - lf[i] * nxt; }
        }
        zc[nb - 1] = cur;
        double x1 = 0.0, x2 = 0.0;
        for (int i = nb - 1; i >= 0; --i) {
          const double xi = (zc[i] - uu[i] * x1 - u2[i] * x2) * rud[i];   // x1 = x2 = 0 past the end
          zc[i] = xi;
          x2 = x1; x1 = xi;
        }
      }
      __syncthreads();
      const int lane = tid & 63, wv = tid >> 6;
      for (int pass = 0; pass < 2; ++pass) {
        // columns k0 .. k - 1 are final and unit-norm: their components of the iterate, one
        // wavefront per column, then all of them removed in one row-wise sweep
        for (int c = k0 + wv; c < k; c += nw) {
          double s = 0.0;
          for (int i = lane; i < nb; i += 64) s += Z[(long)(b0 + i) * ldz + c] * zc[i];
          s = wave_sum(s);
          if (lane == 0) dots[c - k0] = s;
        }
        __syncthreads();
        for (int i = tid; i < nb; i += blockDim.x) {
          const double* zr = Z + (long)(b0 + i) * ldz;
          double acc = 0.0;
          for (int c = k0; c < k; ++c) acc += dots[c - k0] * zr[c];
          zc[i] -= acc;
        }
        __syncthreads();
        double s = 0.0;
        for (int i = tid; i < nb; i += blockDim.x) s += zc[i] * zc[i];
        const double dt = block_sum(s);
        const double sc = (dt > 0.0 && isfinite(dt)) ? 1.0 / sqrt(dt) : 0.0;
        if (sc == 0.0 && tid == 0) atomicOr(status, KFAC_DS_EIG_NOCONV);
        for (int i = tid; i < nb; i += blockDim.x) zc[i] *= sc;
        __syncthreads();
      }
    }
    for (int i = tid; i < nb; i += blockDim.x) Z[(long)(b0 + i) * ldz + k] = zc[i];
    __syncthreads();
  }
}

// Normalise the cluster leaders (columns that start a cluster of size > 1) before the
// member pass projects against them.
__device__ __forceinline__ void tri_cluster_lead_body(const EigTask& q, int, int) {
  const int n = q.n, r = q.r; const TriMeta& m = q.m; double* Z = q.Z; const long ldz = q.ldz;
  __shared__ double red[4];
  __shared__ double sdot;
  if (m.scal[2] == 0.0) return;
  const int tid = threadIdx.x;
  for (int k = 0; k + 1 < r; ++k) {
    if (!(m.cstart[k] && !m.cstart[k + 1])) continue;
    double s = 0.0;
    for (int i = tid; i < n; i += blockDim.x) { const double z = Z[(long)i * ldz + k]; s += z * z; }
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) sdot = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    const double sc = sdot > 0.0 ? 1.0 / sqrt(sdot) : 0.0;
    for (int i = tid; i < n; i += blockDim.x) Z[(long)i * ldz + k] *= sc;
    __syncthreads();
  }
}

// ======================================================================================
// 7. Back-transformation P = H_0 ... H_{n-3} z for each of the first r columns (the column
// is normalised first).  Eight lanes carry one column: lane 8 c + g holds rows 8 u + g
// (u < U) of column c of its wavefront, so a reflector's dot product is eight short sums
// reduced in three DPP steps, and the rows above a chunk's lowest reflector (a prefix of u
// in blocks of 32 rows, the same for every lane) are skipped.  Reflectors are staged in LDS
// in chunks of 16 (8 above width 288; row pitch 8 U, zero beyond n), the next chunk's loads
// in flight while the current one is applied.  fp32 output, rows n..n_pad-1 zero;
// grid = ceil(r / 32) blocks of 256 threads (8 columns per wavefront).
// ======================================================================================
// reflectors per staged chunk (fewer for the widest matrices: registers)
template <int NMAX> constexpr int bt_ch() { return NMAX > kPlanMaxSketch ? 8 : 16; }

__device__ __forceinline__ double bt_colsum(double x) {     // over the column's 8 lanes
  x += dpp_any<0xB1>(x);
  x += dpp_any<0x4E>(x);
  x += dpp_any<0x141>(x);
  return x;
}

// Reflectors k = kt down to klo of the staged chunk on the lane's rows 8 u + g, u >= U0
// (rows below 8 U0 are zero in every reflector of the chunk).
template <int U, int U0>
__device__ __forceinline__ void bt_apply(double (&z)[U], const double* vch, int kt, int klo, int g) {
#pragma unroll 1
  for (int k = kt; k >= klo; --k) {
    const double* vk = vch + (k - klo) * (8 * U) + g;
    double vv[U], s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = U0; u < U; ++u) {
      vv[u] = vk[8 * u];
      s4[u & 3] = fma(vv[u], z[u], s4[u & 3]);
    }
    const double t = 2.0 * bt_colsum((s4[0] + s4[1]) + (s4[2] + s4[3]));
#pragma unroll
    for (int u = U0; u < U; ++u) z[u] = fma(-t, vv[u], z[u]);
  }
}

// Staging of reflector chunks into LDS, the next chunk's loads in registers meanwhile.
template <int NMAX>
struct BtStage {
  static constexpr int CH = bt_ch<NMAX>(), CPT = (CH * NMAX + 255) / 256;
  const double* V;
  int n;
  double* vch;
  double pre[CPT];
  // chunk (reflectors klo .. klo + cnt - 1) into registers: element e = j * NMAX + i is row
  // i of reflector klo + j (zero for i >= n)
  __device__ __forceinline__ void load(int klo, int cnt) {
    const double* src = V + (long)klo * n;
#pragma unroll
    for (int t = 0; t < CPT; ++t) {
      const int e = threadIdx.x + 256 * t, j = e / NMAX, i = e - j * NMAX;
      pre[t] = (j < cnt && i < n) ? src[(long)j * n + i] : 0.0;
    }
  }
  __device__ __forceinline__ void store() {
#pragma unroll
    for (int t = 0; t < CPT; ++t) {
      const int e = threadIdx.x + 256 * t;
      if (e < CH * NMAX) vch[e] = pre[t];
    }
  }
};

// The chunks (from kt down) whose lowest reflector klo has (klo + 1) / 32 == B: their
// rows below 32 B are zero.  kt moves down chunk by chunk; the phases run in decreasing
// B, each a loop of its own, so z stays in the same registers from phase to phase.
template <int U, int B, int NMAX>
__device__ __forceinline__ void bt_phase(double (&z)[U], BtStage<NMAX>& st, int& kt, int g) {
  constexpr int CH = BtStage<NMAX>::CH;
  while (kt >= 0) {
    const int klo = max(0, kt - CH + 1);
    if ((klo + 1) / 32 != B) return;          // uniform
    __syncthreads();                          // the previous chunk's readers are done
    st.store();
    __syncthreads();
    if (kt - CH >= 0) {
      const int nlo = max(0, kt - CH - CH + 1);
      st.load(nlo, kt - CH - nlo + 1);
    }
    bt_apply<U, 4 * B>(z, st.vch, kt, klo, g);
    kt -= CH;
  }
}

template <int U, int NMAX, int... Is>
__device__ __forceinline__ void bt_phases(std::integer_sequence<int, Is...>, double (&z)[U], BtStage<NMAX>& st,
                                          int& kt, int g) {
  constexpr int NB = NMAX / 32;
  (bt_phase<U, NB - 1 - Is, NMAX>(z, st, kt, g), ...);
}

template <int NMAX>
__device__ __forceinline__ void backtransform_body(const EigTask& q, int bx, int) {
  constexpr int U = NMAX / 8;
  static_assert(NMAX % 32 == 0, "row blocks of 32");
  const double* Z = q.Z; const long ldz = q.ldz; const int n = q.n, n_pad = q.n_pad;
  const int r = q.r; float* P = q.P; const long ldp = q.ldp;
  __shared__ double vch[bt_ch<NMAX>() * NMAX];
  BtStage<NMAX> st;
  st.V = q.V; st.n = n; st.vch = vch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane & 7;
  const int c = (bx * 4 + wave) * 8 + (lane >> 3);
  const bool cin = c < r;
  double z[U];
  double nn = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = 8 * u + g;
    z[u] = (cin && i < n) ? Z[(long)i * ldz + c] : 0.0;
    nn = fma(z[u], z[u], nn);
  }
  nn = bt_colsum(nn);
  double sc = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
  if (q.svd && cin) {                        // left singular vectors: W p_k / sigma_k
    const double lk = q.Dd[c];
    sc = (lk > 0.0) ? sc / sqrt(lk) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) z[u] *= sc;
  int kt = n - 3;
  constexpr int CH = BtStage<NMAX>::CH;
  if (kt >= 0) st.load(max(0, kt - CH + 1), kt - max(0, kt - CH + 1) + 1);
  bt_phases(std::make_integer_sequence<int, NMAX / 32>{}, z, st, kt, g);
  if (cin) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = 8 * u + g;
      if (i < n_pad) P[(long)i * ldp + c] = (i < n) ? (float)z[u] : 0.f;
    }
  }
}

// single-task and grouped entry points of the eigensolver phases
__global__ __launch_bounds__(TNT) void k_tridiag_reg(EigTask q) { tridiag_reg_body(q, 0, 0); }
__global__ __launch_bounds__(512) void k_tri_prep(EigTask q) { tri_prep_body(q, 0, 0); }
__global__ __launch_bounds__(256) void k_tri_bisect(EigTask q) { tri_bisect_body(q, blockIdx.x, 0); }
__global__ __launch_bounds__(512) void k_tri_select(EigTask q) { tri_select_body(q, 0, 0); }
template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_tri_vec(EigTask q) { tri_vec_body<NT, NMAX>(q, blockIdx.x, 0); }
__global__ __launch_bounds__(256) void k_tri_cluster_lead(EigTask q) { tri_cluster_lead_body(q, 0, 0); }
__global__ __launch_bounds__(256) void k_tri_cluster(EigTask q) { tri_cluster_body(q, 0, 0); }
template <int NMAX>
__global__ __launch_bounds__(256) void k_backtransform(EigTask q) {
  backtransform_body<NMAX>(q, blockIdx.x, 0);
}

KFAC_GROUPED_KERNEL(k_tridiag_reg_g, tridiag_reg_body, EigTask, TNT)
KFAC_GROUPED_KERNEL(k_tri_prep_g, tri_prep_body, EigTask, 512)
KFAC_GROUPED_KERNEL(k_tri_bisect_g, tri_bisect_body, EigTask, 256)
KFAC_GROUPED_KERNEL(k_tri_select_g, tri_select_body, EigTask, 512)
__global__ __launch_bounds__(32) void k_tri_vec_g(const EigTask* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate(gm, t, bx, by);
  tri_vec_body<32, TNMAX>(tasks[t], bx, by);
}
KFAC_GROUPED_KERNEL(k_tri_cluster_lead_g, tri_cluster_lead_body, EigTask, 256)
KFAC_GROUPED_KERNEL(k_tri_cluster_g, tri_cluster_body, EigTask, 256)
KFAC_GROUPED_KERNEL(k_backtransform_g, backtransform_body<kPlanMaxSketch>, EigTask, 256)

// ======================================================================================
size_t small_eig_scratch_doubles(int n, int r) {
  // es[n] | lam[n] | scal[8] | int blo[n], bhi[n], col_task[r], cstart[r] | cluster[5n]
  return 2 * (size_t)n + 8 + ((size_t)2 * n + 2 * r + 1) / 2 + 2 + 5 * (size_t)n + 16;
}

EigTask make_eig_task(const double* C, long ldc, const float* Cf, long ldcf, int n, int n_pad, int r, double* A,
                      double* V, double* diag, double* off, double* Z, double* scratch, float* P, long ldp, float* D,
                      double* Dd, int* status) {
  // scratch layout (doubles): es[n] | lam[n] | scal[8] | ints blo[n], bhi[n], col_task[r], cstart[r] | cl[5n]
  EigTask q;
  q.C = C; q.ldc = ldc; q.Cf = Cf; q.ldcf = ldcf;
  q.n = n; q.n_pad = n_pad; q.r = r;
  q.A = A; q.V = V; q.diag = diag; q.off = off; q.Z = Z; q.ldz = r;
  double* p = scratch;
  q.m.es = p; p += n;
  q.m.lam = p; p += n;
  q.m.scal = p; p += 8;
  int* ip = (int*)p;
  q.m.blo = ip; ip += n;
  q.m.bhi = ip; ip += n;
  q.m.col_task = ip; ip += r;
  q.m.cstart = ip; ip += r;
  q.cl = (double*)(((uintptr_t)ip + 15) & ~(uintptr_t)15);
  q.P = P; q.ldp = ldp; q.D = D; q.Dd = Dd; q.status = status;
  q.svd = 0;
  return q;
}

hipError_t launch_small_eig(const double* C, long ldc, const float* Cf, long ldcf, int n, int n_pad, int r,
                            double* A, double* V, double* diag, double* off, double* Z, double* scratch,
                            float* P, long ldp, float* D, double* Dd, int* status, hipStream_t s, int svd) {
  EigTask q = make_eig_task(C, ldc, Cf, ldcf, n, n_pad, r, A, V, diag, off, Z, scratch, P, ldp, D, Dd, status);
  q.svd = svd;
  if (n <= TNMAX) hipLaunchKernelGGL(k_tridiag_reg, dim3(1), dim3(TNT), 0, s, q);
  else hipLaunchKernelGGL(k_tridiag_gmem, dim3(1), dim3(1024), 0, s, q);
  hipLaunchKernelGGL(k_tri_prep, dim3(1), dim3(512), 0, s, q);
  hipLaunchKernelGGL(k_tri_bisect, dim3(tri_bisect_blocks(n)), dim3(256), 0, s, q);
  hipLaunchKernelGGL(k_tri_select, dim3(1), dim3(512), 0, s, q);
  if (n <= TNMAX) hipLaunchKernelGGL((k_tri_vec<32, TNMAX>), dim3((r + 31) / 32), dim3(32), 0, s, q);
  else hipLaunchKernelGGL((k_tri_vec<16, KFAC_MAX_SKETCH>), dim3((r + 15) / 16), dim3(16), 0, s, q);
  hipLaunchKernelGGL(k_tri_cluster_lead, dim3(1), dim3(256), 0, s, q);
  hipLaunchKernelGGL(k_tri_cluster, dim3(1), dim3(256), 0, s, q);
  if (n <= kPlanMaxSketch) hipLaunchKernelGGL(k_backtransform<kPlanMaxSketch>, dim3(backtransform_blocks(r)), dim3(256), 0, s, q);
  else hipLaunchKernelGGL(k_backtransform<KFAC_MAX_SKETCH>, dim3(backtransform_blocks(r)), dim3(256), 0, s, q);
  return hipGetLastError();
}

#define KFAC_GLAUNCH(FN, KER, T, NT)                                                         \
  hipError_t FN(const T* tasks, GroupMap gm, int blocks, hipStream_t s) {                  \
    if (blocks > 0) hipLaunchKernelGGL(KER, dim3(blocks), dim3(NT), 0, s, tasks, gm);      \
    return hipGetLastError();                                                              \
  }
KFAC_GLAUNCH(launch_tridiag_g, k_tridiag_reg_g, EigTask, TNT)
KFAC_GLAUNCH(launch_tri_prep_g, k_tri_prep_g, EigTask, 512)
KFAC_GLAUNCH(launch_tri_bisect_g, k_tri_bisect_g, EigTask, 256)
KFAC_GLAUNCH(launch_tri_select_g, k_tri_select_g, EigTask, 512)
KFAC_GLAUNCH(launch_tri_vec_g, k_tri_vec_g, EigTask, 32)
KFAC_GLAUNCH(launch_tri_cluster_lead_g, k_tri_cluster_lead_g, EigTask, 256)
KFAC_GLAUNCH(launch_tri_cluster_g, k_tri_cluster_g, EigTask, 256)
KFAC_GLAUNCH(launch_backtransform_g, k_backtransform_g, EigTask, 256)
int tri_bisect_blocks(int n) { return (n + BIS_PER_BLOCK - 1) / BIS_PER_BLOCK; }
int tri_vec_blocks(int r) { return (r + 31) / 32; }
int backtransform_blocks(int r) { return (r + 31) / 32; }
}  // namespace kfac
