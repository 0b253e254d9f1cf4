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

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
struct TileF32 {
  static constexpr int NT = WM * WN * kWave;
  static constexpr int FM = BM / WM / 16;
  static constexpr int FN = BN / WN / 16;
  static constexpr int SA = BM + lds_pad(BM);
  static constexpr int SB = BN + lds_pad(BN);
  static constexpr int LA = BM * BK / NT;
  static constexpr int LB = BN * BK / NT;
  static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "tile/wave shape");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "loader shape");
  static_assert(BK % 4 == 0, "BK multiple of 4");
  struct Smem {
    float a[BK][SA];
    float b[BK][SB];
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

  __device__ static __forceinline__ void fetch(const GemmP& p, int m0, int n0, int k0, int kend,
                                               float ra[LA], float rb[LB]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      int e = t + i * NT, m, k;
      if (TA) { k = e / BM; m = e % BM; } else { m = e / BK; k = e % BK; }
      ra[i] = (k0 + k < kend) ? ldA(p, m0 + m, k0 + k) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      int e = t + i * NT, n, k;
      if (TB) { n = e / BK; k = e % BK; } else { k = e / BN; n = e % BN; }
      rb[i] = (k0 + k < kend) ? ldB(p, k0 + k, n0 + n) : 0.f;
    }
  }
  __device__ static __forceinline__ void stash(Smem& sm, const float ra[LA], const float rb[LB]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      int e = t + i * NT, m, k;
      if (TA) { k = e / BM; m = e % BM; } else { m = e / BK; k = e % BK; }
      sm.a[k][m] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      int e = t + i * NT, n, k;
      if (TB) { n = e / BK; k = e % BK; } else { k = e / BN; n = e % BN; }
      sm.b[k][n] = rb[i];
    }
  }

  // acc += A[m0:m0+BM, kb:ke] * B[kb:ke, n0:n0+BN]
  __device__ static void run(const GemmP& p, int m0, int n0, int kb, int ke, Smem& sm,
                             f32x4 acc[FM][FN]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int am = wm * (BM / WM) + (lane & 15), bn = wn * (BN / WN) + (lane & 15);
    const int kq = lane >> 4;
    float ra[LA], rb[LB];
    if (kb >= ke) return;
    fetch(p, m0, n0, kb, ke, ra, rb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
      __syncthreads();
      stash(sm, ra, rb);
      __syncthreads();
      if (k0 + BK < ke) fetch(p, m0, n0, k0 + BK, ke, ra, rb);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[i] = sm.a[kk + kq][am + i * 16];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[j] = sm.b[kk + kq][bn + j * 16];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
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

}  // namespace kfac
