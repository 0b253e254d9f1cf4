// fp32 kernels of the K-factor pipeline: identity init, the generic MFMA GEMM with its
// epilogues, the symmetric EA update (Alg. 1 EA lines) with split-K, the Gaussian test
// matrix (Alg. 2/3 "Sample Gaussian Matrix") and the column sign convention of U.
#include "kernels.h"
#include "conv.h"

namespace kfac {

// ------------------------------------------------------------------------------------
__global__ void k_fill_identity(float* F, int d, long ldf) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)d * d;
  for (; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx / d), j = (int)(idx % d);
    F[(long)i * ldf + j] = (i == j) ? 1.f : 0.f;
  }
}

// ------------------------------------------------------------------------------------
// Generic GEMM body (gemm_tile_body in gemm_f32.h) on fp32 MFMA tiles.
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT = false>
__device__ __forceinline__ void gemm_body(const GemmP& p, int bx, int by) {
  gemm_tile_body<TileF32<BM, BN, BK, WM, WN, TA, TB>, SPLIT>(p, bx, by);
}

// Split-K finish: 1024 consecutive elements of C per block; slices summed in index order,
// then the GEMM's epilogue.
constexpr int kGemmSliceChunk = 1024;
__device__ __forceinline__ void gemm_slices_body(const GemmP& p, int bx, int) {
  const long total = (long)p.M * p.N;
  for (int u = 0; u < kGemmSliceChunk / 256; ++u) {
    const long e = (long)bx * kGemmSliceChunk + u * 256 + threadIdx.x;
    if (e >= total) return;
    float v = 0.f;
    for (int sl = 0; sl < p.ksplit; ++sl) v += p.part[(long)sl * total + e];
    const int i = (int)(e / p.N), j = (int)(e % p.N);
    float s = p.alpha * v;
    if (p.rowD) s *= damp_weight(p.rowD[i], p.lam);
    if (p.colD) s *= damp_weight(p.colD[j], p.lam);
    if (p.X) s += p.beta * p.X[(long)i * p.ldx + j];
    p.C[(long)i * p.ldc + j] = s;
    if (p.Cb) p.Cb[(long)i * p.ldcb + j] = f32_to_bf16_rne(s);
  }
}
KFAC_GROUPED_KERNEL(k_gemm_slices_g, gemm_slices_body, GemmP, 256)

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(WM * WN * 64) void k_gemm(GemmP p) {
  gemm_body<BM, BN, BK, WM, WN, TA, TB>(p, blockIdx.x, blockIdx.y);
}

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT = false>
__global__ __launch_bounds__(WM * WN * 64) void k_gemm_g(const GemmP* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate(gm, t, bx, by);
  gemm_body<BM, BN, BK, WM, WN, TA, TB, SPLIT>(tasks[t], bx, by);
}

// ------------------------------------------------------------------------------------
// EA update F <- rho F + c * Xh^T Xh on upper-triangular BT x BT tiles.
// A = Xh^T (stored K x M: TA), B = Xh (stored K x N).
constexpr int EA_BT = 64, EA_BK = 16, EA_WM = 2, EA_WN = 2;
using EaTile = TileF32<EA_BT, EA_BT, EA_BK, EA_WM, EA_WN, true, false>;

union EaSmem {
  EaTile::Smem g;
  float t[EA_BT][EA_BT + 1];
};

__device__ __forceinline__ void ea_tiles_body(const EaTask& q, int bx, int by) {
  __shared__ EaSmem sm;
  const GemmP& p = q.g;
  int I, J;
  ea_tile(bx, q.T, I, J);
  const int ks = by, nks = q.nks;
  int kb, ke;
  ea_slice(p.K, nks, ks, EA_BK, kb, ke);
  f32x4 acc[EaTile::FM][EaTile::FN];
#pragma unroll
  for (int i = 0; i < EaTile::FM; ++i)
#pragma unroll
    for (int j = 0; j < EaTile::FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  EaTile::run(p, I * EA_BT, J * EA_BT, kb, ke, sm.g, acc);
  if (nks > 1) {
    float* slot = p.part + ((long)bx * nks + ks) * (EA_BT * EA_BT);
    EaTile::for_each(acc, [&](int r, int c, float v) { slot[r * EA_BT + c] = v; });
    return;
  }
  __syncthreads();
  EaTile::for_each(acc, [&](int r, int c, float v) { sm.t[r][c] = v; });
  __syncthreads();
  ea_store_tile_t<EA_BT>(sm.t, q.o, I, J);
}

// Deterministic split-K reduction (slices summed in index order) + EA epilogue, one
// 16-row chunk of a tile per block.
__device__ __forceinline__ void ea_finalize_body(const EaTask& q, int bx, int) {
  __shared__ float v[kEaChunk][EA_BT + 1];
  ea_finalize_chunk<EA_BT>(q, bx, v);
}

__global__ __launch_bounds__(256) void k_ea_tiles(EaTask q) {
  const int l = xcd_swizzle(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  ea_tiles_body(q, l % gridDim.x, l / gridDim.x);
}
__global__ __launch_bounds__(256) void k_ea_finalize(EaTask q) { ea_finalize_body(q, blockIdx.x, 0); }
__global__ __launch_bounds__(256) void k_ea_tiles_g(const EaTask* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate_xcd8(gm, t, bx, by);
  if (by >= tasks[t].nks) return;
  ea_tiles_body(tasks[t], bx, by);
}
KFAC_GROUPED_KERNEL(k_ea_finalize_g, ea_finalize_body, EaTask, 256)

// F <- rho F (n == 0), keeps the bf16 shadow in sync.
__global__ void k_scale_factor(float* F, long ldf, uint16_t* Fb, long ldfb, int d, float rho) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)d * d;
  for (; idx < total; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx / d), j = (int)(idx % d);
    float v = rho * F[(long)i * ldf + j];
    F[(long)i * ldf + j] = v;
    if (Fb) Fb[(long)i * ldfb + j] = f32_to_bf16_rne(v);
  }
}

// ------------------------------------------------------------------------------------
// Gaussian test matrix.  Thread (row i, group g) draws columns 4g..4g+3.
// Transposed workspace form: OmT[j][i] (rows j < l_pad, ld = ldt), zero outside d x l.
// User form: Om[i][j] with ldo, plus optional raw words.  Block (bx, by) = (row block,
// column group).
__device__ __forceinline__ void omega_body(const OmegaTask& p, int bx, int by) {
  const int i = bx * blockDim.x + threadIdx.x;
  const int g = by;
  const int rows = p.d_pad > p.d ? p.d_pad : p.d;
  if (i >= rows) return;
  double z[4] = {0, 0, 0, 0};
  uint32_t w[4] = {0, 0, 0, 0};
  const bool live = i < p.d;
  if (live) gaussian4((uint32_t)i, (uint32_t)g, p.stream, p.inv, p.k0, p.k1, z, w);
  const int groups = (p.l + 3) / 4;
  if (live && p.words && g < groups) {
#pragma unroll
    for (int t = 0; t < 4; ++t) p.words[((long)i * groups + g) * 4 + t] = w[t];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = 4 * g + t;
    const float v = (live && j < p.l) ? (float)z[t] : 0.f;
    if (p.OmT && j < p.l_pad) p.OmT[(long)j * p.ldt + i] = v;
    if (p.OmTb && j < p.l_pad) p.OmTb[(long)j * p.ldt + i] = f32_to_bf16_rne(v);
    if (p.Om && live && j < p.l) p.Om[(long)i * p.ldo + j] = v;
  }
}

__global__ void k_omega(OmegaTask p) { omega_body(p, blockIdx.x, blockIdx.y); }
KFAC_GROUPED_KERNEL(k_omega_g, omega_body, OmegaTask, 256)

// ------------------------------------------------------------------------------------
// Sign convention: the largest-magnitude entry of each column of U is made positive
// (ties: lowest row).  Phase 1: per 256-row chunk and column, the (first) entry of
// largest magnitude, kept with its sign.  Phase 2: every block derives the column signs
// from the chunk partials (in chunk order) and flips its own chunk.
// Block = 256 threads = 4 row groups x 64 columns; grid (ceil(r/64), ceil(d/256)).
constexpr int SG_ROWS = 256;

__device__ __forceinline__ void sign_partial_body(const SignTask& q, int bx, int by) {
  float* U = q.U; const long ldu = q.ldu; const int d = q.d, r = q.r; float* pval = q.pval; int* pidx = q.pidx;
  __shared__ float sv[4][64];
  __shared__ int si[4][64];
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int c = bx * 64 + cl, chunk = by;
  const int r0 = chunk * SG_ROWS, r1 = min(d, r0 + SG_ROWS);
  float best = -1.f, bval = 0.f;
  int bidx = 0x7fffffff;
  if (c < r) {
#pragma unroll 8
    for (int i = r0 + rg; i < r1; i += 4) {
      const float v = U[(long)i * ldu + c];
      if (fabsf(v) > best) { best = fabsf(v); bval = v; bidx = i; }
    }
  }
  sv[rg][cl] = bval; si[rg][cl] = bidx;
  __syncthreads();
  if (rg == 0 && c < r) {
    float bv = sv[0][cl];
    int bi = si[0][cl];
    for (int g = 1; g < 4; ++g) {
      const float v = sv[g][cl];
      const int vi = si[g][cl];
      if (fabsf(v) > fabsf(bv) || (fabsf(v) == fabsf(bv) && vi < bi)) { bv = v; bi = vi; }
    }
    pval[(long)chunk * r + c] = bv;
    pidx[(long)chunk * r + c] = bi;
  }
}

__device__ __forceinline__ void sign_apply_body(const SignTask& q, int bx, int by) {
  float* U = q.U; const long ldu = q.ldu; const int d = q.d, r = q.r, nchunks = q.nchunks;
  const float* pval = q.pval; const int* pidx = q.pidx;
  __shared__ float ssgn[64];
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int c = bx * 64 + cl, chunk = by;
  if (rg == 0) {
    float s = 1.f;
    if (c < r) {
      float bv = 0.f;
      int bi = 0x7fffffff;
      for (int k = 0; k < nchunks; ++k) {
        const float v = pval[(long)k * r + c];
        const int vi = pidx[(long)k * r + c];
        if (fabsf(v) > fabsf(bv) || (fabsf(v) == fabsf(bv) && vi < bi)) { bv = v; bi = vi; }
      }
      s = (bv < 0.f) ? -1.f : 1.f;
    }
    ssgn[cl] = s;
  }
  __syncthreads();
  if (c >= r || ssgn[cl] > 0.f) return;
  const int r0 = chunk * SG_ROWS, r1 = min(d, r0 + SG_ROWS);
#pragma unroll 8
  for (int i = r0 + rg; i < r1; i += 4) U[(long)i * ldu + c] = -U[(long)i * ldu + c];
}

__global__ __launch_bounds__(256) void k_sign_partial(SignTask q) { sign_partial_body(q, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(256) void k_sign_apply(SignTask q) { sign_apply_body(q, blockIdx.x, blockIdx.y); }
KFAC_GROUPED_KERNEL(k_sign_partial_g, sign_partial_body, SignTask, 256)
KFAC_GROUPED_KERNEL(k_sign_apply_g, sign_apply_body, SignTask, 256)

// ------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------
hipError_t launch_fill_identity(float* F, int d, long ldf, hipStream_t s) {
  long total = (long)d * d;
  int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_identity, dim3(blocks), dim3(256), 0, s, F, d, ldf);
  return hipGetLastError();
}

template <bool TA, bool TB>
static hipError_t gemm_dispatch(const GemmP& p, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  if (p.M >= 128 && p.N >= 128 && (long)p.M * p.N >= 128L * 128 * 256) {
    dim3 grid((p.N + 127) / 128, (p.M + 127) / 128);
    hipLaunchKernelGGL((k_gemm<128, 128, 16, 2, 2, TA, TB>), grid, dim3(256), 0, s, p);
  } else {
    dim3 grid((p.N + 63) / 64, (p.M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<64, 64, 16, 2, 2, TA, TB>), grid, dim3(256), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmP& p, bool ta, bool tb, hipStream_t s) {
  if (!ta && !tb) return gemm_dispatch<false, false>(p, s);
  if (!ta && tb) return gemm_dispatch<false, true>(p, s);
  if (ta && !tb) return gemm_dispatch<true, false>(p, s);
  return gemm_dispatch<true, true>(p, s);
}

int ea_tiles_per_side(int d, bool bf) {
  const int bt = bf ? kEaBf16Tile : EA_BT;
  return (d + bt - 1) / bt;
}

int ea_choose_ksplit(int d, long n, bool bf) {
  const int T = ea_tiles_per_side(d, bf);
  const long tiles = (long)T * (T + 1) / 2;
  // Split-K count from a simple cost model: the tiles run in rounds of `slots` resident
  // workgroups (two per compute unit for bf16, four for fp32), a round lasting as long
  // as one slice; each slice adds a tile of partial sums written and read back.
  const long slots = bf ? 512 : 1024;
  const long rows = bf ? 1024 : 512;                // rows per slice at least
  const long maxk = std::max<long>(1, std::min<long>(64, (n + rows - 1) / rows));
  const double stage_us = bf ? 1.6 : 1.2;           // one 64- / 32-row step of a block
  const double step_rows = bf ? 64.0 : 32.0;
  const double tile_us = (double)(bf ? kEaBf16Tile : EA_BT) * (bf ? kEaBf16Tile : EA_BT) * 8.0 / 8e6;
  long best = 1;
  double best_cost = 0.0;
  for (long ks = 1; ks <= maxk; ++ks) {
    const long rounds = (tiles * ks + slots - 1) / slots;
    double cost = (double)rounds * ((double)n / ks / step_rows) * stage_us;
    if (ks > 1) cost += (double)(tiles * ks) * tile_us + 5.0;
    if (ks == 1 || cost < best_cost) { best = ks; best_cost = cost; }
  }
  return (int)best;
}

size_t ea_partial_bytes(int d, int ks, bool bf) {
  if (ks <= 1) return 0;
  const long bt = bf ? kEaBf16Tile : EA_BT;
  const long T = ea_tiles_per_side(d, bf);
  return (size_t)(T * (T + 1) / 2) * ks * bt * bt * sizeof(float);
}

int ea_grouped_ksplit(int d, long n, bool bf, double total_steps) {
  // In a grouped launch every slice of every factor is one workgroup of the same grid:
  // slices only have to keep the longest workgroup well below the launch's length.
  const double slots = bf ? 512.0 : 1024.0, step_rows = bf ? 64.0 : 32.0;
  const double smax = std::max(32.0, total_steps / slots / 3.0);
  const long rows = bf ? 1024 : 512;
  const long maxk = std::max<long>(1, std::min<long>(64, (n + rows - 1) / rows));
  const long ks = (long)std::ceil(std::ceil((double)n / step_rows) / smax);
  return (int)std::max<long>(1, std::min<long>(ks, maxk));
}

size_t ea_workspace_bytes(int d, long n, bool bf) {
  int ks = ea_choose_ksplit(d, n, bf);
  if (ks <= 1) return 0;
  const long bt = bf ? kEaBf16Tile : EA_BT;
  int T = ea_tiles_per_side(d, bf);
  long tiles = (long)T * (T + 1) / 2;
  return (size_t)tiles * ks * bt * bt * sizeof(float);
}

int ea_finalize_chunks(bool bf) { return (bf ? kEaBf16Tile : EA_BT) / kEaChunk; }

size_t ea_workspace_bytes(int d, long n) {
  return std::max(ea_workspace_bytes(d, n, false), ea_workspace_bytes(d, n, true));
}

static hipError_t launch_ea_common(float* F, int d, long ldf, const float* X, const uint16_t* Xb, int n,
                                   int d_in, long ldx, int ones, float rho, float scale, uint16_t* Fb, long ldfb,
                                   void* ws, size_t ws_bytes, hipStream_t s, const ConvGeom* cv = nullptr) {
  if (n == 0) {
    long total = (long)d * d;
    int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_scale_factor, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, F, ldf, Fb,
                       ldfb, d, rho);
    return hipGetLastError();
  }
  const bool bf = (Xb != nullptr);
  int ks = ea_choose_ksplit(d, n, bf);
  if (ks > 1 && (ws == nullptr || ws_bytes < ea_workspace_bytes(d, n, bf))) ks = 1;
  EaTask q = make_ea_task(F, d, ldf, X, Xb, n, d_in, ldx, ones, rho, scale, Fb, ldfb, (float*)ws, ks);
  if (cv) q.cv = *cv;
  const int tiles = q.T * (q.T + 1) / 2;
  if (bf) {
    hipError_t e = launch_ea_bf16_tiles(q, tiles, ks, s);
    if (e != hipSuccess || ks == 1) return e;
    return launch_ea_bf16_finalize(q, tiles, s);
  }
  hipLaunchKernelGGL(k_ea_tiles, dim3(tiles, ks), dim3(256), 0, s, q);
  if (ks > 1) hipLaunchKernelGGL(k_ea_finalize, dim3(tiles * ea_finalize_chunks(false)), dim3(256), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_ea_f32(float* F, int d, long ldf, const float* X, int n, int d_in, long ldx,
                         int ones, float rho, float scale, uint16_t* Fb, long ldfb, void* ws,
                         size_t ws_bytes, hipStream_t s) {
  return launch_ea_common(F, d, ldf, X, nullptr, n, d_in, ldx, ones, rho, scale, Fb, ldfb, ws, ws_bytes, s);
}

hipError_t launch_ea_bf16(float* F, int d, long ldf, const uint16_t* X, int n, int d_in, long ldx, int ones,
                          float rho, float scale, uint16_t* Fb, long ldfb, void* ws, size_t ws_bytes,
                          hipStream_t s) {
  return launch_ea_common(F, d, ldf, nullptr, X, n, d_in, ldx, ones, rho, scale, Fb, ldfb, ws, ws_bytes, s);
}

hipError_t launch_ea_bf16_conv(float* F, int d, long ldf, const uint16_t* x, const ConvGeom& cv, int ones, float rho,
                               float scale, uint16_t* Fb, long ldfb, void* ws, size_t ws_bytes, hipStream_t s) {
  const int n = cv.B * cv.Ho * cv.Wo, d_in = cv.kh * cv.kw * cv.C;
  const size_t pb = conv_patch_bytes(cv, true);
  if (pb > 0 && ws && (((uintptr_t)ws) & 15) == 0 && ws_bytes >= pb && n > 0) {
    uint16_t* P = (uint16_t*)ws;
    const int ldp = conv_patch_ld(cv);
    hipError_t e = launch_im2col_stage(x, cv, P, ldp, n, s);
    if (e != hipSuccess) return e;
    return launch_ea_common(F, d, ldf, nullptr, P, n, d_in, ldp, ones, rho, scale, Fb, ldfb, (char*)ws + pb,
                            ws_bytes - pb, s);
  }
  return launch_ea_common(F, d, ldf, nullptr, x, n, d_in, 0, ones, rho, scale, Fb, ldfb, ws, ws_bytes, s, &cv);
}

OmegaTask make_omega_task(int d, int l, int d_pad, int l_pad, uint64_t seed, uint64_t stream_id, uint32_t inv,
                          float* OmT, long ldt, uint16_t* OmTb, float* Om, long ldo, uint32_t* words) {
  OmegaTask p;
  p.d = d; p.l = l; p.d_pad = d_pad; p.l_pad = l_pad;
  p.k0 = (uint32_t)(seed & 0xffffffffu); p.k1 = (uint32_t)(seed >> 32);
  p.stream = (uint32_t)(stream_id & 0xffffffffu); p.inv = inv;
  p.OmT = OmT; p.ldt = ldt; p.OmTb = OmTb; p.Om = Om; p.ldo = ldo; p.words = words;
  return p;
}

dim3 omega_grid(const OmegaTask& p) {
  const int rows = p.d_pad > p.d ? p.d_pad : p.d;
  const int groups = std::max((p.l + 3) / 4, (p.l_pad + 3) / 4);
  return dim3((rows + 255) / 256, groups);
}

hipError_t launch_omega(int d, int l, int d_pad, int l_pad, uint64_t seed, uint64_t stream_id,
                        uint32_t inv, float* OmT, long ldt, uint16_t* OmTb, float* Om, long ldo,
                        uint32_t* words, hipStream_t s) {
  OmegaTask p = make_omega_task(d, l, d_pad, l_pad, seed, stream_id, inv, OmT, ldt, OmTb, Om, ldo, words);
  hipLaunchKernelGGL(k_omega, omega_grid(p), dim3(256), 0, s, p);
  return hipGetLastError();
}

int sign_chunks(int d) { return (d + SG_ROWS - 1) / SG_ROWS; }

hipError_t launch_sign_normalize(float* U, long ldu, int d, int r, float* pval, int* pidx, hipStream_t s) {
  SignTask q{U, ldu, d, r, pval, pidx, sign_chunks(d)};
  dim3 grid((r + 63) / 64, sign_chunks(d));
  hipLaunchKernelGGL(k_sign_partial, grid, dim3(256), 0, s, q);
  hipLaunchKernelGGL(k_sign_apply, grid, dim3(256), 0, s, q);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// grouped launchers
#define KFAC_GLAUNCH(FN, KER, T, NT)                                                         \
  hipError_t FN(const T* tasks, GroupMap gm, int blocks, hipStream_t s) {                  \
    if (blocks > 0) hipLaunchKernelGGL(KER, dim3(blocks), dim3(NT), 0, s, tasks, gm);      \
    return hipGetLastError();                                                              \
  }
KFAC_GLAUNCH(launch_ea_tiles_g, k_ea_tiles_g, EaTask, 256)
KFAC_GLAUNCH(launch_ea_finalize_g, k_ea_finalize_g, EaTask, 256)
KFAC_GLAUNCH(launch_omega_g, k_omega_g, OmegaTask, 256)
KFAC_GLAUNCH(launch_sign_partial_g, k_sign_partial_g, SignTask, 256)
KFAC_GLAUNCH(launch_sign_apply_g, k_sign_apply_g, SignTask, 256)

// Skinny fp32 GEMM for the Rayleigh-Ritz product W = F Q of Alg. 3 (stored transposed,
// W^T = Q^T F): C[M x N] = A[M x K] B[K x N] with M <= 288 (the sketch width), A K-contiguous,
// B N-contiguous.  A workgroup owns all M rows and 64 columns over the whole K, so F is read
// once; 8 wavefronts as 2 (M) x 4 (N), each 144 x 16 (9 MFMA tiles); BK = 16, two LDS
// buffers.
constexpr int SF_M = 288, SF_BN = 64, SF_BK = 16, SF_NT = 512;
constexpr int SF_SA = SF_M + lds_pad(SF_M), SF_SB = SF_BN + lds_pad(SF_BN);
struct alignas(16) SfSmem {
  float a[2][SF_BK][SF_SA];
  float b[2][SF_BK][SF_SB];
};
constexpr int SF_GA = (SF_M * SF_BK / 4 + SF_NT - 1) / SF_NT;       // float4 groups per thread
constexpr int SF_GB = (SF_BN * SF_BK / 4 + SF_NT - 1) / SF_NT;

__device__ __forceinline__ void gemm_skinny_f32_body(const GemmP& p, int bx, int) {
  __shared__ SfSmem sm;
  const int n0 = bx * SF_BN;
  const int M = p.M, N = p.N, K = p.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mt = (M + 15) / 16;
  const bool va = ((p.lda & 3) == 0) && ((((uintptr_t)p.A) & 15) == 0);
  const bool vb = ((p.ldb & 3) == 0) && ((((uintptr_t)p.B) & 15) == 0);
  f32x4 acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  // two register stages: the loads of k-step s+2 are issued while step s computes
  float4 ra[2][SF_GA], rb[2][SF_GB];
  auto fetch = [&](int k0, float4 (&xa)[SF_GA], float4 (&xb)[SF_GB]) {
#pragma unroll
    for (int u = 0; u < SF_GA; ++u) {
      const int g = tid + u * SF_NT;
      const int m = g / (SF_BK / 4), k = (g % (SF_BK / 4)) * 4, gk = k0 + k;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < SF_M * SF_BK / 4 && m < M) {
        const float* src = p.A + (long)m * p.lda + gk;
        if (va && gk + 4 <= K) v = *(const float4*)src;
        else {
          v.x = (gk < K) ? src[0] : 0.f; v.y = (gk + 1 < K) ? src[1] : 0.f;
          v.z = (gk + 2 < K) ? src[2] : 0.f; v.w = (gk + 3 < K) ? src[3] : 0.f;
        }
      }
      xa[u] = v;
    }
#pragma unroll
    for (int u = 0; u < SF_GB; ++u) {
      const int g = tid + u * SF_NT;
      const int k = g / (SF_BN / 4), n = (g % (SF_BN / 4)) * 4, gk = k0 + k, gn = n0 + n;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < SF_BN * SF_BK / 4 && gk < K) {
        const float* src = p.B + (long)gk * p.ldb + gn;
        if (vb && gn + 4 <= N) v = *(const float4*)src;
        else {
          v.x = (gn < N) ? src[0] : 0.f; v.y = (gn + 1 < N) ? src[1] : 0.f;
          v.z = (gn + 2 < N) ? src[2] : 0.f; v.w = (gn + 3 < N) ? src[3] : 0.f;
        }
      }
      xb[u] = v;
    }
  };
  auto stash = [&](int buf, const float4 (&xa)[SF_GA], const float4 (&xb)[SF_GB]) {
#pragma unroll
    for (int u = 0; u < SF_GA; ++u) {
      const int g = tid + u * SF_NT;
      if (g >= SF_M * SF_BK / 4) continue;
      const int m = g / (SF_BK / 4), k = (g % (SF_BK / 4)) * 4;
      const int rot = (k >> 2) & 3;                  // spread one store over four k-rows
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = (i + rot) & 3;
        sm.a[buf][k + j][m] = f4_elem(xa[u], j);
      }
    }
#pragma unroll
    for (int u = 0; u < SF_GB; ++u) {
      const int g = tid + u * SF_NT;
      if (g >= SF_BN * SF_BK / 4) continue;
      const int k = g / (SF_BN / 4), n = (g % (SF_BN / 4)) * 4;
      *(float4*)&sm.b[buf][k][n] = xb[u];
    }
  };
  const int nsteps = (K + SF_BK - 1) / SF_BK;
  if (nsteps > 0) {
    fetch(0, ra[0], rb[0]);
    stash(0, ra[0], rb[0]);
    if (nsteps > 1) fetch(SF_BK, ra[1], rb[1]);
    __syncthreads();
  }
  for (int s = 0; s < nsteps; ++s) {
    const int cur = s & 1, nxt = cur ^ 1;
    // registers [cur] held step s (already in LDS); reuse them for step s + 2
    if (s + 2 < nsteps) {
      if (cur == 0) fetch((s + 2) * SF_BK, ra[0], rb[0]);
      else fetch((s + 2) * SF_BK, ra[1], rb[1]);
    }
    // all operand reads of the k-step first (one LDS latency per step), then the MFMAs
    float af[SF_BK / 4][9], bfv[SF_BK / 4];
#pragma unroll
    for (int u = 0; u < SF_BK / 4; ++u) {
      const int kq = 4 * u + (lane >> 4);
      bfv[u] = sm.b[cur][kq][wn * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 9; ++i) af[u][i] = sm.a[cur][kq][wm * 144 + i * 16 + (lane & 15)];
    }
#pragma unroll
    for (int u = 0; u < SF_BK / 4; ++u)
#pragma unroll
      for (int i = 0; i < 9; ++i)
        if (wm * 9 + i < mt)                          // uniform: skip m tiles beyond M
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[u][i], bfv[u], acc[i], 0, 0, 0);
    // registers [nxt] hold step s + 1: into the other LDS buffer
    if (s + 1 < nsteps) {
      if (nxt == 0) stash(0, ra[0], rb[0]);
      else stash(1, ra[1], rb[1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wm * 144 + i * 16 + 4 * (lane >> 4) + r;
      const int col = n0 + wn * 16 + (lane & 15);
      if (row >= M || col >= N) continue;
      float v = p.alpha * acc[i][r];
      if (p.rowD) v *= damp_weight(p.rowD[row], p.lam);
      if (p.colD) v *= damp_weight(p.colD[col], p.lam);
      if (p.X) v += p.beta * p.X[(long)row * p.ldx + col];
      p.C[(long)row * p.ldc + col] = v;
      if (p.Cb) p.Cb[(long)row * p.ldcb + col] = f32_to_bf16_rne(v);
    }
}
KFAC_GROUPED_KERNEL_XCD(k_gemm_skinny_f32_g, gemm_skinny_f32_body, GemmP, SF_NT)

// Tile configurations of the grouped fp32 GEMM (BM x BN, 2 x 2 wavefronts, BK = 16).
template <int BM, int BN>
static void gemm_g_launch(const GemmP* tasks, GroupMap gm, int blocks, bool ta, bool tb, bool split, hipStream_t s) {
  if (split) hipLaunchKernelGGL((k_gemm_g<BM, BN, 16, 2, 2, false, false, true>), dim3(blocks), dim3(256), 0, s, tasks, gm);
  else if (!ta && !tb) hipLaunchKernelGGL((k_gemm_g<BM, BN, 16, 2, 2, false, false>), dim3(blocks), dim3(256), 0, s, tasks, gm);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm_g<BM, BN, 16, 2, 2, false, true>), dim3(blocks), dim3(256), 0, s, tasks, gm);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm_g<BM, BN, 16, 2, 2, true, false>), dim3(blocks), dim3(256), 0, s, tasks, gm);
  else hipLaunchKernelGGL((k_gemm_g<BM, BN, 16, 2, 2, true, true>), dim3(blocks), dim3(256), 0, s, tasks, gm);
}

static const int kGemmCfg[kGemmConfigs][2] = {{64, 64}, {128, 128}, {96, 128}, {128, 64}, {SF_M, SF_BN}};

hipError_t launch_gemm_g(const GemmP* tasks, GroupMap gm, int blocks, bool ta, bool tb, int cfg, bool split,
                         hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (split && (ta || tb || cfg == 4)) return hipErrorInvalidValue;   // split-K: plain layouts, square tiles
  switch (cfg) {
    case 1: gemm_g_launch<128, 128>(tasks, gm, blocks, ta, tb, split, s); break;
    case 2: gemm_g_launch<96, 128>(tasks, gm, blocks, ta, tb, split, s); break;
    case 3: gemm_g_launch<128, 64>(tasks, gm, blocks, ta, tb, split, s); break;
    case 4:   // skinny: no transposes, M <= 288 (checked by the caller)
      if (ta || tb) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_gemm_skinny_f32_g, dim3(blocks), dim3(SF_NT), 0, s, tasks, gm);
      break;
    default: gemm_g_launch<64, 64>(tasks, gm, blocks, ta, tb, split, s); break;
  }
  return hipGetLastError();
}
int gemm_g_blocks_x(const GemmP& p, int cfg) { return (p.N + kGemmCfg[cfg][1] - 1) / kGemmCfg[cfg][1]; }
int gemm_g_blocks_y(const GemmP& p, int cfg) {
  return (p.M + kGemmCfg[cfg][0] - 1) / kGemmCfg[cfg][0] * (p.ksplit > 1 ? p.ksplit : 1);
}
int gemm_slice_blocks(const GemmP& p) {
  return p.ksplit > 1 ? (int)(((long)p.M * p.N + kGemmSliceChunk - 1) / kGemmSliceChunk) : 0;
}
hipError_t launch_gemm_slices_g(const GemmP* tasks, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_gemm_slices_g, dim3(blocks), dim3(256), 0, s, tasks, gm);
  return hipGetLastError();
}
int precondition_ksplit(int64_t d_g, int64_t d_a, int64_t r_a) {
  // T1 = J U_a diag(f_a) (d_g x r_a, contraction over d_a): few 64 x 64 tiles, long K
  const int64_t tiles = ((d_g + 63) / 64) * ((r_a + 63) / 64);
  const int64_t want = (256 + tiles - 1) / tiles, maxk = (d_a + 511) / 512;
  return (int)std::max<int64_t>(1, std::min<int64_t>({want, maxk, (int64_t)16}));
}

EaTask make_ea_task(float* F, int d, long ldf, const float* X, const uint16_t* Xb, int n, int d_in, long ldx, int ones,
                    float rho, float scale, uint16_t* Fb, long ldfb, float* part, int ks) {
  EaOut o{F, ldf, Fb, ldfb, d, rho, (1.f - rho) * scale};
  GemmP p{};
  p.M = d; p.N = d; p.K = n;
  p.A = X; p.lda = ldx; p.B = X; p.ldb = ldx;
  p.Ab = Xb; p.Bb = Xb;
  p.ones_col = ones ? d_in : -1;
  p.ksplit = ks;
  p.part = part;
  EaTask q{p, o, ea_tiles_per_side(d, Xb != nullptr), ks};
  return q;
}

}  // namespace kfac
