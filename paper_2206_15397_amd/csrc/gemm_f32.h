// FP32 tiled GEMM on gfx950 MFMA (v_mfma_f32_16x16x4_f32), C = op(A) op(B), with the
// epilogues the K-factor pipeline needs.  Operand tiles are staged through LDS in
// K-major order (smem[k][m], smem[k][n]) so each 16-lane group of a wavefront reads 16
// consecutive words; the row pitch is padded so the four k-rows read by one wavefront
// land in distinct banks.
#pragma once
#include "common.h"

namespace kfac {

enum Epi : int {
  EPI_GENERAL = 0,   // C = alpha*acc*rs[i]*cs[j] + beta*X ; optional bf16 copy
  EPI_PARTIAL = 1,   // raw tile -> split-K workspace slot
  EPI_EA = 2         // symmetric EA blend, mirrored, optional bf16 shadow
};

struct GemmP {
  int M, N, K;
  const float* A; long lda;     // TA ? A is K x M : A is M x K   (row-major)
  const float* B; long ldb;     // TB ? B is N x K : B is K x N
  float* C; long ldc;
  float alpha, beta;
  const float* X; long ldx;     // EPI_GENERAL additive term (may be null)
  const float* rowD;            // EPI_GENERAL: row scale f(rowD[i]) = 1/(D+lam) - 1/lam
  const float* colD;            //              col scale likewise
  float lam;
  uint16_t* Cb; long ldcb;      // optional bf16 copy of C
  int ones_col;                 // EA: column index of the appended ones (or -1)
  float* part;                  // EPI_PARTIAL workspace base
  int ksplit;                   // number of K slices (gridDim.y)
  float rho, ea_c;              // EA: F <- rho F + ea_c * acc
  const uint16_t* Ab;           // if set, A is read as bf16 (same layout as A)
  const uint16_t* Bb;           // if set, B is read as bf16
};

__host__ __device__ constexpr int lds_pad(int bm) { return ((16 - bm) % 64 + 64) % 64; }

// Element j (run-time, 0..3) of a float4, by selects (no dynamic register indexing).
__device__ __forceinline__ float f4_elem(const float4& v, int j) {
  const float a = (j & 1) ? v.y : v.x;
  const float b = (j & 1) ? v.w : v.z;
  return (j & 2) ? b : a;
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
struct TileF32 {
  static constexpr int BM_ = BM, BN_ = BN, BK_ = BK;
  static constexpr int NT = WM * WN * kWave;
  static constexpr int FM = BM / WM / 16;
  static constexpr int FN = BN / WN / 16;
  static constexpr int SA = BM + lds_pad(BM);
  static constexpr int SB = BN + lds_pad(BN);
  static constexpr int LA = BM * BK / NT;       // elements per thread and k-step
  static constexpr int LB = BN * BK / NT;
  // groups of 4 memory-contiguous elements per thread (the last round may be partial)
  static constexpr int NGA = BM * BK / 4, NGB = BN * BK / 4;
  static constexpr int GA = (NGA + NT - 1) / NT, GB = (NGB + NT - 1) / NT;
  static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "tile/wave shape");
  static_assert(BM % 4 == 0 && BN % 4 == 0, "loader shape");
  static_assert(BK % 4 == 0, "BK multiple of 4");
  struct alignas(16) Smem {
    float a[2][BK][SA];
    float b[2][BK][SB];
  };

  __device__ static __forceinline__ float ldA(const GemmP& p, int m, int k) {
    if (m >= p.M || k >= p.K) return 0.f;
    if (m == p.ones_col) return 1.f;
    long o = TA ? (long)k * p.lda + m : (long)m * p.lda + k;
    return p.Ab ? bf16_to_f32(p.Ab[o]) : p.A[o];
  }
  __device__ static __forceinline__ float ldB(const GemmP& p, int k, int n) {
    if (n >= p.N || k >= p.K) return 0.f;
    if (n == p.ones_col) return 1.f;
    long o = TB ? (long)n * p.ldb + k : (long)k * p.ldb + n;
    return p.Bb ? bf16_to_f32(p.Bb[o]) : p.B[o];
  }
  // Group g of an operand tile: (row index along M or N, k) of its first element; the four
  // elements run along the operand's memory-contiguous dimension.
  __device__ static __forceinline__ void a_group(int g, int& m, int& k) {
    if (TA) { k = g / (BM / 4); m = (g % (BM / 4)) * 4; } else { m = g / (BK / 4); k = (g % (BK / 4)) * 4; }
  }
  __device__ static __forceinline__ void b_group(int g, int& n, int& k) {
    if (TB) { n = g / (BK / 4); k = (g % (BK / 4)) * 4; } else { k = g / (BN / 4); n = (g % (BN / 4)) * 4; }
  }

  __device__ static __forceinline__ void fetch(const GemmP& p, int m0, int n0, int k0, int kend, bool va, bool vb,
                                               float4 ra[GA], float4 rb[GB]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < GA; ++u) {
      int m, k;
      if (t + u * NT >= NGA) { ra[u] = make_float4(0.f, 0.f, 0.f, 0.f); continue; }
      a_group(t + u * NT, m, k);
      const int gm = m0 + m, gk = k0 + k;
      // 16-byte load when the four elements are in range, aligned and not the ones column
      const bool full = TA ? (gm + 4 <= p.M && gk < kend && (p.ones_col < gm || p.ones_col >= gm + 4))
                           : (gm < p.M && gk + 4 <= kend && gm != p.ones_col);
      if (va && full) {
        ra[u] = *(const float4*)(p.A + (TA ? (long)gk * p.lda + gm : (long)gm * p.lda + gk));
      } else {
        float e[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int mm = TA ? gm + i : gm, kk = TA ? gk : gk + i;
          e[i] = (kk < kend) ? ldA(p, mm, kk) : 0.f;
        }
        ra[u] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
#pragma unroll
    for (int u = 0; u < GB; ++u) {
      int n, k;
      if (t + u * NT >= NGB) { rb[u] = make_float4(0.f, 0.f, 0.f, 0.f); continue; }
      b_group(t + u * NT, n, k);
      const int gn = n0 + n, gk = k0 + k;
      const bool full = TB ? (gn < p.N && gk + 4 <= kend && gn != p.ones_col)
                           : (gn + 4 <= p.N && gk < kend && (p.ones_col < gn || p.ones_col >= gn + 4));
      if (vb && full) {
        rb[u] = *(const float4*)(p.B + (TB ? (long)gn * p.ldb + gk : (long)gk * p.ldb + gn));
      } else {
        float e[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int nn = TB ? gn : gn + i, kk = TB ? gk + i : gk;
          e[i] = (kk < kend) ? ldB(p, kk, nn) : 0.f;
        }
        rb[u] = make_float4(e[0], e[1], e[2], e[3]);
      }
    }
  }
  __device__ static __forceinline__ void stash(Smem& sm, int buf, const float4 ra[GA], const float4 rb[GB]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < GA; ++u) {
      int m, k;
      if (t + u * NT >= NGA) continue;
      a_group(t + u * NT, m, k);
      if (TA) {
        *(float4*)&sm.a[buf][k][m] = ra[u];          // four consecutive m: one 16-byte store
      } else {
        // four consecutive k of one m: rotate the order by k/4 so the lanes of one store
        // hit four different k-rows (bank groups) instead of the same one
        const int rot = (k >> 2) & 3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = (i + rot) & 3;
          sm.a[buf][k + j][m] = f4_elem(ra[u], j);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < GB; ++u) {
      int n, k;
      if (t + u * NT >= NGB) continue;
      b_group(t + u * NT, n, k);
      if (!TB) {
        *(float4*)&sm.b[buf][k][n] = rb[u];
      } else {
        const int rot = (k >> 2) & 3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = (i + rot) & 3;
          sm.b[buf][k + j][n] = f4_elem(rb[u], j);
        }
      }
    }
  }

  // acc += A[m0:m0+BM, kb:ke] * B[kb:ke, n0:n0+BN]; two LDS buffers, one barrier per k-step.
  __device__ static __forceinline__ void run(const GemmP& p, int m0, int n0, int kb, int ke, Smem& sm, f32x4 acc[FM][FN]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int am = wm * (BM / WM) + (lane & 15), bn = wn * (BN / WN) + (lane & 15);
    const int kq = lane >> 4;
    if (kb >= ke) return;
    const bool va = !p.Ab && ((p.lda & 3) == 0) && ((((uintptr_t)p.A) & 15) == 0);
    const bool vb = !p.Bb && ((p.ldb & 3) == 0) && ((((uintptr_t)p.B) & 15) == 0);
    float4 ra[GA], rb[GB];
    fetch(p, m0, n0, kb, ke, va, vb, ra, rb);
    __syncthreads();                 // the caller's LDS may alias ours (unions)
    stash(sm, 0, ra, rb);
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) fetch(p, m0, n0, k0 + BK, ke, va, vb, ra, rb);
      // all operand reads of the k-step first (one LDS latency per step), then the MFMAs
      float af[BK / 4][FM], bf[BK / 4][FN];
#pragma unroll
      for (int u = 0; u < BK / 4; ++u) {
#pragma unroll
        for (int i = 0; i < FM; ++i) af[u][i] = sm.a[buf][4 * u + kq][am + i * 16];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[u][j] = sm.b[buf][4 * u + kq][bn + j * 16];
      }
#pragma unroll
      for (int u = 0; u < BK / 4; ++u)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[u][i], bf[u][j], acc[i][j], 0, 0, 0);
      if (more) stash(sm, buf ^ 1, ra, rb);
      __syncthreads();
      buf ^= 1;
    }
  }

  // Visit every accumulator element with its (row, col) inside the BM x BN tile.
  template <typename Fn>
  __device__ static __forceinline__ void for_each(f32x4 acc[FM][FN], Fn&& fn) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int row = wm * (BM / WM) + i * 16 + 4 * (lane >> 4) + r;
          int col = wn * (BN / WN) + j * 16 + (lane & 15);
          fn(row, col, acc[i][j][r]);
        }
  }
};

__device__ __forceinline__ float damp_weight(float D, float lam) {
  return 1.0f / (D + lam) - 1.0f / lam;
}

// (I, J) of the t-th upper-triangular tile, row-major over I <= J, T tiles per side.
__device__ __forceinline__ void upper_tile(int t, int T, int& I, int& J) {
  int i = 0, rem = t;
  while (rem >= T - i) { rem -= T - i; ++i; }
  I = i; J = i + rem;
}

// Generic GEMM on tile type T (TileF32): block (bx, by) computes
// C[by*BM : , bx*BN : ].  With ksplit > 1, by also names the K slice (by = slice * tile rows
// + tile row) and the raw tile goes to slice `slice` of the partial sums (ksplit x M x N,
// row-major), to be finished by the slice-reduction kernel, which applies the epilogue.
template <typename T, bool SPLIT = false>
__device__ __forceinline__ void gemm_tile_body(const GemmP& p, int bx, int by) {
  constexpr int BM = T::BM_, BN = T::BN_, BK = T::BK_;
  __shared__ typename T::Smem sm;
  int kb = 0, ke = p.K, slice = 0;
  if constexpr (SPLIT) {
    if (p.ksplit > 1) {
      const int ty = (p.M + BM - 1) / BM;
      slice = by / ty;
      by -= slice * ty;
      const int kc = ((p.K + p.ksplit - 1) / p.ksplit + BK - 1) / BK * BK;
      kb = min(p.K, slice * kc);
      ke = min(p.K, kb + kc);
    }
  }
  const int m0 = by * BM, n0 = bx * BN;
  f32x4 acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  T::run(p, m0, n0, kb, ke, sm, acc);
  if (SPLIT && p.ksplit > 1) {
    float* part = p.part + (long)slice * p.M * p.N;
    T::for_each(acc, [&](int r, int c, float v) {
      const int i = m0 + r, j = n0 + c;
      if (i < p.M && j < p.N) part[(long)i * p.N + j] = v;
    });
    return;
  }
  T::for_each(acc, [&](int r, int c, float v) {
    int i = m0 + r, j = n0 + c;
    if (i >= p.M || j >= p.N) return;
    float s = p.alpha * v;
    if (p.rowD) s *= damp_weight(p.rowD[i], p.lam);
    if (p.colD) s *= damp_weight(p.colD[j], p.lam);
    if (p.X) s += p.beta * p.X[(long)i * p.ldx + j];
    p.C[(long)i * p.ldc + j] = s;
    if (p.Cb) p.Cb[(long)i * p.ldcb + j] = f32_to_bf16_rne(s);
  });
}

}  // namespace kfac
