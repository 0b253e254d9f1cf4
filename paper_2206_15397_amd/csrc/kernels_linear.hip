// K-FAC linear layer on bf16 MFMA (fp32 accumulation):
//   forward   y = x W^T + b                         (A = x, B = W, both K-contiguous)
//   backward  dx = g W                              (A = g K-contiguous, B = W K-major)
//             [dW | db] = g^T [x | 1]               (both operands K-major: batch rows)
//             Gamma <- rho Gamma + (1 - rho) s g^T g  (the backward-factor EA of Alg. 1, fused
//                                                     into the same launch as dW: the g
//                                                     columns it reads are the dW tiles' A)
// 128 x 128 tiles, 4 waves of 64 x 64 on v_mfma_f32_16x16x32_bf16, 64-deep k-steps with two
// LDS buffers.  Operands whose contraction index is the row index (K-major) are loaded as
// 8 x 8 blocks and transposed in registers, so LDS always holds k-contiguous rows.
#include "kernels.h"
#include "conv.h"

namespace kfac {

constexpr int LN_T = 128, LN_BK = 64, LN_SK = LN_BK + 8;

struct alignas(16) LinSmem {
  union {
    struct {
      uint16_t a[2][LN_T][LN_SK];
      uint16_t b[2][LN_T][LN_SK];
    } g;
    float t[LN_T][LN_T + 1];
  };
};

// Column c of the row-major 8 x 8 bf16 block v[row].
__device__ __forceinline__ uint4 ln_col_of_block(const uint4 v[8], int c) {
  auto half = [&](int r) -> uint32_t {
    const uint4& x = v[r];
    const uint32_t w = (c >> 1) == 0 ? x.x : (c >> 1) == 1 ? x.y : (c >> 1) == 2 ? x.z : x.w;
    return (c & 1) ? (w >> 16) : (w & 0xffffu);
  };
  return make_uint4(half(0) | (half(1) << 16), half(2) | (half(3) << 16), half(4) | (half(5) << 16),
                    half(6) | (half(7) << 16));
}

// Rows [k0, k0+8) x columns [c0, c0+8) of a K-major operand with `cols` stored columns and an
// optional ones column at index `cols` (zero beyond, and beyond row K).
__device__ __forceinline__ void ln_load_kmajor(const uint16_t* X, long ld, int cols, bool ones, bool vec, int k0,
                                               int K, int c0, uint4 v[8]) {
  const bool full = vec && (c0 + 8 <= cols);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = k0 + r;
    v[r] = make_uint4(0, 0, 0, 0);
    if (k >= K) continue;
    const uint16_t* p = X + (long)k * ld + c0;
    if (full) {
      v[r] = *(const uint4*)p;
    } else {
      uint16_t t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = c0 + j;
        t[j] = (c < cols) ? p[j] : ((ones && c == cols) ? (uint16_t)0x3f80 : (uint16_t)0);
      }
      v[r] = make_uint4(t[0] | ((uint32_t)t[1] << 16), t[2] | ((uint32_t)t[3] << 16),
                        t[4] | ((uint32_t)t[5] << 16), t[6] | ((uint32_t)t[7] << 16));
    }
  }
}

// 16 bytes (8 k-values) of row `row` of a K-contiguous operand.
__device__ __forceinline__ uint4 ln_ld16(const uint16_t* base, long ld, int row, int nrows, int k, int K, bool vec) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row < nrows) {
    const uint16_t* p = base + (long)row * ld + k;
    if (vec && k + 8 <= K) {
      v = *(const uint4*)p;
    } else {
      uint16_t t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = (k + i < K) ? p[i] : (uint16_t)0;
      v = make_uint4(t[0] | ((uint32_t)t[1] << 16), t[2] | ((uint32_t)t[3] << 16), t[4] | ((uint32_t)t[5] << 16),
                     t[6] | ((uint32_t)t[7] << 16));
    }
  }
  return v;
}

// One operand tile (128 rows of M or N by 64 k) per k-step, filled by 128 threads.
struct LnOperand {
  const uint16_t* X; long ld;
  int rows;        // M or N extent (K-contiguous) / stored columns (K-major)
  bool ones;       // K-major: implicit ones column at index `rows`
  bool vec;        // 16-byte loads allowed
  ConvGeom cv;     // K-major, C > 0: X is an NHWC input read as its im2col patches
};

// CONV: 0, or the im2col loader form (1: 16-byte, 2: element loads) of a K-major operand
// that may be im2col patches (o.cv.C > 0, decided per operand at run time)
template <bool KMAJ, int CONV = 0>
struct LnLoader {
  uint4 v[8];
  __device__ __forceinline__ void load(const LnOperand& o, int tt, int r0, int k0, int K) {
    if (KMAJ) {
      const int cg = tt >> 3, rg = tt & 7;
      if (CONV != 0 && o.cv.C > 0) im2col_block<CONV>(o.X, o.cv, o.ones, k0 + rg * 8, K, r0 + cg * 8, v);
      else ln_load_kmajor(o.X, o.ld, o.rows, o.ones, o.vec, k0 + rg * 8, K, r0 + cg * 8, v);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tt + 128 * u, row = e >> 3, kc = (e & 7) * 8;
        v[u] = ln_ld16(o.X, o.ld, r0 + row, o.rows, k0 + kc, K, o.vec);
      }
    }
  }
  __device__ __forceinline__ void store(uint16_t (*dst)[LN_SK], int tt) {
    if (KMAJ) {
      const int cg = tt >> 3, rg = tt & 7;
#pragma unroll
      for (int c = 0; c < 8; ++c) *(uint4*)&dst[cg * 8 + c][rg * 8] = ln_col_of_block(v, c);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tt + 128 * u, row = e >> 3, kc = (e & 7) * 8;
        *(uint4*)&dst[row][kc] = v[u];
      }
    }
  }
};

__device__ __forceinline__ bool ln_vec_ok(const uint16_t* X, long ld) {
  return ((ld & 7) == 0) && ((((uintptr_t)X) & 15) == 0);
}

// Block bx of a LinTask.  AK / BK: operand stored K-major (rows = contraction index).
template <bool AK, bool BK, int CONV = 0>
__device__ __forceinline__ void lin_body(const LinTask& q, int bx, int ks = 0) {
  __shared__ LinSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int nplain = q.tiles_m * q.tiles_n;
  const bool gam = bx >= nplain;
  int m0, n0, GI = 0, GJ = 0;
  LnOperand oa{q.A, q.lda, q.M, false, ln_vec_ok(q.A, q.lda), ConvGeom{}};
  LnOperand ob{q.B, q.ldb, BK ? (q.b_ones ? q.N - 1 : q.N) : q.N, BK && q.b_ones != 0, ln_vec_ok(q.B, q.ldb),
               CONV ? q.cv : ConvGeom{}};
  if (!gam) {
    m0 = (bx % q.tiles_m) * LN_T;
    n0 = (bx / q.tiles_m) * LN_T;
  } else {
    ea_tile(bx - nplain, q.gam_T, GI, GJ);
    m0 = GI * LN_T;
    n0 = GJ * LN_T;
    ob = oa;                       // g^T g: both operands are g's columns
  }
  const bool same = gam && GI == GJ;
  // contraction rows [kb, K) of this K slice (the whole contraction when nks == 1)
  int kb = 0, K = q.K;
  if (q.nks > 1) ea_slice(q.K, q.nks, ks, LN_BK, kb, K);
  const int op = tid >> 7, tt = tid & 127;
  const bool loader = !(same && op == 1);
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // one register set per thread: threads 0-127 fill the A tile, 128-255 the B tile (with
  // equal layouts a single loader object, so its registers are never selected at run time)
  LnLoader<AK, CONV> la;
  LnLoader<BK, CONV> lb;
  auto fetch = [&](int k0) {
    if (!loader) return;
    if constexpr (AK == BK) {
      la.load(op ? ob : oa, tt, op ? n0 : m0, k0, K);
    } else {
      if (op == 0) la.load(oa, tt, m0, k0, K);
      else lb.load(ob, tt, n0, k0, K);
    }
  };
  auto stash = [&](int buf) {
    if (!loader) return;
    if constexpr (AK == BK) {
      la.store(op ? sm.g.b[buf] : sm.g.a[buf], tt);
    } else {
      if (op == 0) la.store(sm.g.a[buf], tt);
      else lb.store(sm.g.b[buf], tt);
    }
  };
  if (kb < K) {
    fetch(kb);
    stash(0);
    __syncthreads();
  }
  int buf = 0;
  for (int k0 = kb; k0 < K; k0 += LN_BK) {
    const bool more = k0 + LN_BK < K;
    if (more) fetch(k0 + LN_BK);
    uint16_t (*As)[LN_SK] = sm.g.a[buf];
    uint16_t (*Bs)[LN_SK] = same ? sm.g.a[buf] : sm.g.b[buf];
#pragma unroll
    for (int kk = 0; kk < LN_BK; kk += 32) {
      const int kq = kk + (lane >> 4) * 8;
      bf16x8 af[4], bfr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&As[wm * 64 + i * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bfr[j] = __builtin_bit_cast(bf16x8, *(const uint4*)&Bs[wn * 64 + j * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (q.nks > 1) {
    // raw sums of this slice; the reduce launch sums the slices in order
    float* slot = q.part + ((long)bx * q.nks + ks) * (LN_T * LN_T);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          slot[(wm * 64 + i * 16 + 4 * (lane >> 4) + r) * LN_T + wn * 64 + j * 16 + (lane & 15)] = acc[i][j][r];
    return;
  }
  if (gam) {
    // backward-factor EA tile: stage raw sums, blend, write tile + mirror + bf16 shadow
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sm.t[wm * 64 + i * 16 + 4 * (lane >> 4) + r][wn * 64 + j * 16 + (lane & 15)] = acc[i][j][r];
    __syncthreads();
    ea_store_tile_t<LN_T>(sm.t, q.gam, GI, GJ);
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < q.M && col < q.N) {
          const float v = acc[i][j][r] + (q.bias ? q.bias[col] : 0.f);
          if (q.C) q.C[(long)row * q.ldc + col] = v;
          if (q.Cb) q.Cb[(long)row * q.ldcb + col] = f32_to_bf16_rne(v);
        }
      }
}

__global__ __launch_bounds__(256) void k_lin_nt(LinTask q) { lin_body<false, false>(q, blockIdx.x); }
__global__ __launch_bounds__(256) void k_lin_nn(LinTask q) { lin_body<false, true>(q, blockIdx.x); }
__global__ __launch_bounds__(256) void k_lin_tn(LinTask q) { lin_body<true, true>(q, blockIdx.x); }
template <int FORM>
__global__ __launch_bounds__(256) void k_lin_tn_conv(LinTask q) {
  lin_body<true, true, FORM>(q, blockIdx.x, blockIdx.y);
}

// Split-K reduce of the weight-gradient launch: block = (tile, 16-row chunk).  Plain tiles:
// C rows [a0, a0 + 16) of the tile = the slices summed in index order.  Fused gam tiles:
// the EA finalize (slices in order, blend, tile + mirror + bf16 shadow).
constexpr int LN_CH = LN_T / kEaChunk;
__global__ __launch_bounds__(256) void k_lin_tn_reduce(LinTask q) {
  __shared__ float v[kEaChunk][LN_T + 1];
  const int nplain = q.tiles_m * q.tiles_n;
  const int tile = blockIdx.x / LN_CH, a0 = (blockIdx.x % LN_CH) * kEaChunk;
  if (tile >= nplain) {
    EaTask e{};
    e.o = q.gam;
    e.T = q.gam_T;
    e.nks = q.nks;
    e.g.part = q.part + (long)nplain * q.nks * (LN_T * LN_T);
    ea_finalize_chunk<LN_T>(e, blockIdx.x - nplain * LN_CH, v);
    return;
  }
  const int m0 = (tile % q.tiles_m) * LN_T, n0 = (tile / q.tiles_m) * LN_T;
  const float* base = q.part + (long)tile * q.nks * (LN_T * LN_T) + (long)a0 * LN_T;
  for (int e = threadIdx.x; e < kEaChunk * LN_T; e += blockDim.x) {
    float s = 0.f;
#pragma unroll 8
    for (int k = 0; k < q.nks; ++k) s += base[(long)k * LN_T * LN_T + e];
    const int row = m0 + a0 + e / LN_T, col = n0 + e % LN_T;
    if (row < q.M && col < q.N) q.C[(long)row * q.ldc + col] = s;
  }
}

static LinTask lin_task(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb, int b_ones,
                        float* C, long ldc, uint16_t* Cb, long ldcb, const float* bias) {
  LinTask q{};
  q.M = M; q.N = N; q.K = K;
  q.A = A; q.lda = lda; q.B = B; q.ldb = ldb; q.b_ones = b_ones;
  q.C = C; q.ldc = ldc; q.Cb = Cb; q.ldcb = ldcb; q.bias = bias;
  q.tiles_m = (M + LN_T - 1) / LN_T;
  q.tiles_n = (N + LN_T - 1) / LN_T;
  q.gam_T = 0;
  q.nks = 1;
  q.part = nullptr;
  return q;
}

hipError_t launch_linear_forward(const uint16_t* x, int n, int d_in, long ldx, const uint16_t* W, int d_out, long ldw,
                                 const float* bias, uint16_t* y, long ldy, hipStream_t s) {
  LinTask q = lin_task(n, d_out, d_in, x, ldx, W, ldw, 0, nullptr, 0, y, ldy, bias);
  const int blocks = q.tiles_m * q.tiles_n;
  if (blocks > 0) hipLaunchKernelGGL(k_lin_nt, dim3(blocks), dim3(256), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_linear_backward(const uint16_t* g, int n, int d_out, long ldg, const uint16_t* x, int d_in, long ldx,
                                  const uint16_t* W, long ldw, uint16_t* dx, long lddx, float* dWb, long lddw,
                                  int with_bias, float* Gam, long ldgam, uint16_t* Gamb, long ldgb, float rho,
                                  float scale, hipStream_t s) {
  if (dx) {
    // dx[n x d_in] = g[n x d_out] W[d_out x d_in]
    LinTask q = lin_task(n, d_in, d_out, g, ldg, W, ldw, 0, nullptr, 0, dx, lddx, nullptr);
    const int blocks = q.tiles_m * q.tiles_n;
    if (blocks > 0) hipLaunchKernelGGL(k_lin_nn, dim3(blocks), dim3(256), 0, s, q);
  }
  // [dW | db][d_out x (d_in + 1)] = g^T [x | 1], plus the upper tiles of g^T g for Gamma
  const int N = d_in + (with_bias ? 1 : 0);
  LinTask q = lin_task(d_out, N, n, g, ldg, x, ldx, with_bias, dWb, lddw, nullptr, 0, nullptr);
  int blocks = q.tiles_m * q.tiles_n;
  if (Gam) {
    q.gam = EaOut{Gam, ldgam, Gamb, ldgb, d_out, rho, (1.f - rho) * scale};
    q.gam_T = q.tiles_m;
    blocks += q.gam_T * (q.gam_T + 1) / 2;
  }
  if (blocks > 0) hipLaunchKernelGGL(k_lin_tn, dim3(blocks), dim3(256), 0, s, q);
  return hipGetLastError();
}

// Tiles of the weight-gradient launch (plain dW tiles + the fused gam tiles) and its K
// slices: enough workgroups to fill the chip twice over, each slice at least four 64-row
// steps; bounded by the workspace (ws_bytes / per-slice bytes).
static int conv_dw_tiles(int c_out, int N) {
  const int tm = (c_out + LN_T - 1) / LN_T, tn = (N + LN_T - 1) / LN_T;
  return tm * tn + tm * (tm + 1) / 2;
}
// At most 64 slices: the slice reduce (and the fused EA finalize, 8 elements per thread)
// sums every slice serially, so hundreds of slices over a few tiles (the first VGG16_bn
// convolution: 256 over 2 tiles) cost more than they save (conv weight gradients 1034 ->
// 945 us with 64 at most; 32 measured slower again).
static int conv_dw_slices(int tiles, long n) {
  const long want = (512 + tiles - 1) / tiles;
  const long most = std::max<long>(1, n / (4 * LN_BK));
  return (int)std::max<long>(1, std::min<long>(std::min(want, most), 64));
}
size_t conv_backward_weight_ws_bytes(int c_out, long n, int N) {
  const int tiles = conv_dw_tiles(c_out, N);
  const int nks = conv_dw_slices(tiles, n);
  return nks > 1 ? (size_t)tiles * nks * LN_T * LN_T * sizeof(float) : 0;
}

hipError_t launch_conv_backward_weight(const uint16_t* g, const uint16_t* x, const ConvGeom& cv, int c_out,
                                       float* dWb, long lddw, int with_bias, float* Gam, long ldgam, uint16_t* Gamb,
                                       long ldgb, float rho, float scale, void* ws, size_t ws_bytes, hipStream_t s) {
  // [dW | db][c_out x (kh kw C + 1)] = g^T [P | 1]: A = g (n x c_out, K-major), B = the patches
  // P (n x kh kw C, K-major, gathered from x), plus the upper tiles of g^T g for Gamma
  const int n = cv.B * cv.Ho * cv.Wo;
  const int N = cv.kh * cv.kw * cv.C + (with_bias ? 1 : 0);
  // staged patches (conv_patch_bytes) at the start of the workspace: B becomes a plain K-major
  // operand (cv.C = 0 selects the ordinary loader), the slices use the rest
  const uint16_t* Bop = x;
  long ldb = 0;
  ConvGeom cvq = cv;
  const size_t pb = conv_patch_bytes(cv, false);
  if (pb > 0 && ws && (((uintptr_t)ws) & 15) == 0 && ws_bytes >= pb && n > 0) {
    const int ldp = conv_patch_ld(cv);
    hipError_t e = launch_im2col_stage(x, cv, (uint16_t*)ws, ldp, n, s);
    if (e != hipSuccess) return e;
    Bop = (const uint16_t*)ws;
    ldb = ldp;
    cvq.C = 0;
    ws = (char*)ws + pb;
    ws_bytes -= pb;
  }
  LinTask q = lin_task(c_out, N, n, g, c_out, Bop, ldb, with_bias, dWb, lddw, nullptr, 0, nullptr);
  q.cv = cvq;
  int blocks = q.tiles_m * q.tiles_n;
  if (Gam) {
    q.gam = EaOut{Gam, ldgam, Gamb, ldgb, c_out, rho, (1.f - rho) * scale};
    q.gam_T = q.tiles_m;
    blocks += q.gam_T * (q.gam_T + 1) / 2;
  }
  if (blocks <= 0) return hipSuccess;
  int nks = ws ? conv_dw_slices(conv_dw_tiles(c_out, N), n) : 1;
  const size_t per_slice = (size_t)blocks * LN_T * LN_T * sizeof(float);
  if (nks > 1) nks = (int)std::min<size_t>(nks, ws_bytes / per_slice);
  if (nks > 1) {
    q.nks = nks;
    q.part = (float*)ws;
    if (cv.vec) hipLaunchKernelGGL(k_lin_tn_conv<1>, dim3(blocks, nks), dim3(256), 0, s, q);
    else hipLaunchKernelGGL(k_lin_tn_conv<2>, dim3(blocks, nks), dim3(256), 0, s, q);
    hipLaunchKernelGGL(k_lin_tn_reduce, dim3(blocks * LN_CH), dim3(256), 0, s, q);
  } else {
    if (cv.vec) hipLaunchKernelGGL(k_lin_tn_conv<1>, dim3(blocks), dim3(256), 0, s, q);
    else hipLaunchKernelGGL(k_lin_tn_conv<2>, dim3(blocks), dim3(256), 0, s, q);
  }
  return hipGetLastError();
}

}  // namespace kfac
