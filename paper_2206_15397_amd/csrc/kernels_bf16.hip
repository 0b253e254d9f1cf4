// bf16 kernels: the sketch / power-iteration product of Alg. 3 in bf16 with fp32
// accumulation (v_mfma_f32_16x16x32_bf16), and the EA update for bf16 activations.
#include "kernels.h"

namespace kfac {

// C[M x N] = A[M x K] * B[N x K]^T ; A, B bf16 row-major, K contiguous; C fp32.
// Tiles BM x BN x 32, 4 waves (2 x 2).  LDS rows hold 32 k-values + 8 pad (80 bytes),
// each lane reads its 8 consecutive k (16 bytes) of one row per fragment.
template <int BM, int BN>
struct TileBF16 {
  static constexpr int BK = 32, PAD = 8, SK = BK + PAD;
  static constexpr int FM = BM / 2 / 16, FN = BN / 2 / 16;
  static constexpr int NT = 256;
  static constexpr int NVA = BM * BK / 8, NVB = BN * BK / 8;   // 16-byte vectors per tile
  static constexpr int VA = (NVA + NT - 1) / NT;                 // per thread (last guarded)
  static constexpr int VB = (NVB + NT - 1) / NT;
  struct Smem {
    uint16_t a[BM][SK];
    uint16_t b[BN][SK];
  };
};

__device__ __forceinline__ uint4 ld16(const uint16_t* base, long ld, int row, int nrows, int k, int K) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row < nrows) {
    const uint16_t* p = base + (long)row * ld + k;
    if (k + 8 <= K && (((uintptr_t)p) & 15) == 0) {
      v = *(const uint4*)p;
    } else {
      uint16_t t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = (k + i < K) ? p[i] : (uint16_t)0;
      v.x = t[0] | ((uint32_t)t[1] << 16); v.y = t[2] | ((uint32_t)t[3] << 16);
      v.z = t[4] | ((uint32_t)t[5] << 16); v.w = t[6] | ((uint32_t)t[7] << 16);
    }
  }
  return v;
}

template <int BM, int BN>
__device__ __forceinline__ void gemm_bf16_body(const BfGemmTask& q, int bx, int) {
  using T = TileBF16<BM, BN>;
  __shared__ typename T::Smem sm;
  const int M = q.M, N = q.N, K = q.K, tiles_m = q.tiles_m;
  const uint16_t* A = q.A; const uint16_t* B = q.B;
  const long lda = q.lda, ldb = q.ldb, ldc = q.ldc;
  float* C = q.C;
  const int tm = bx % tiles_m, tn = bx / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f32x4 acc[T::FM][T::FN];
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ra[T::VA], rb[T::VB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < T::VA; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      ra[u] = (e < T::NVA) ? ld16(A, lda, m0 + row, M, k0 + kc, K) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < T::VB; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      rb[u] = (e < T::NVB) ? ld16(B, ldb, n0 + row, N, k0 + kc, K) : make_uint4(0, 0, 0, 0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += T::BK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < T::VA; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      if (e < T::NVA) *(uint4*)&sm.a[row][kc] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < T::VB; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      if (e < T::NVB) *(uint4*)&sm.b[row][kc] = rb[u];
    }
    __syncthreads();
    if (k0 + T::BK < K) fetch(k0 + T::BK);
    const int kq = (lane >> 4) * 8;
    bf16x8 af[T::FM], bfr[T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i) {
      uint4 v = *(const uint4*)&sm.a[wm * (BM / 2) + i * 16 + (lane & 15)][kq];
      af[i] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int j = 0; j < T::FN; ++j) {
      uint4 v = *(const uint4*)&sm.b[wn * (BN / 2) + j * 16 + (lane & 15)][kq];
      bfr[j] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
        int col = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
        if (row < M && col < N) C[(long)row * ldc + col] = acc[i][j][r];
      }
}

constexpr int BF_BM = 96, BF_BN = 128;
__global__ __launch_bounds__(256) void k_gemm_bf16_nt(BfGemmTask q) { gemm_bf16_body<BF_BM, BF_BN>(q, blockIdx.x, 0); }
__global__ __launch_bounds__(256) void k_gemm_bf16_nt_g(const BfGemmTask* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate(gm, t, bx, by);
  gemm_bf16_body<BF_BM, BF_BN>(tasks[t], bx, by);
}

BfGemmTask make_bf16_task(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb, float* C,
                          long ldc) {
  BfGemmTask q{M, N, K, A, lda, B, ldb, C, ldc, (M + BF_BM - 1) / BF_BM};
  return q;
}
int bf16_task_blocks(const BfGemmTask& q) { return q.tiles_m * ((q.N + BF_BN - 1) / BF_BN); }

hipError_t launch_gemm_bf16_nt(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb,
                               float* C, long ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  BfGemmTask q = make_bf16_task(M, N, K, A, lda, B, ldb, C, ldc);
  hipLaunchKernelGGL(k_gemm_bf16_nt, dim3(bf16_task_blocks(q)), dim3(256), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16_g(const BfGemmTask* tasks, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_gemm_bf16_nt_g, dim3(blocks), dim3(256), 0, s, tasks, gm);
  return hipGetLastError();
}
}  // namespace kfac
