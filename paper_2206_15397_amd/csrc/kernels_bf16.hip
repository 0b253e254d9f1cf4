// bf16 kernels: the sketch / power-iteration product of Alg. 3 in bf16 with fp32
// accumulation (v_mfma_f32_16x16x32_bf16), and the EA update for bf16 activations.
#include "kernels.h"
#include "conv.h"

namespace kfac {

// C[M x N] = A[M x K] * B[N x K]^T ; A, B bf16 row-major, K contiguous; C fp32.
// Tiles BM x BN x 64, 4 waves (2 x 2), two LDS buffers (one barrier per k-step).  LDS rows
// hold 64 k-values + 8 pad (144 bytes), so the 16 rows read by one 16-lane group fall on
// distinct banks; each lane reads its 8 consecutive k (16 bytes) of one row per operand.
template <int BM, int BN>
struct TileBF16 {
  static constexpr int BK = 64, PAD = 8, SK = BK + PAD;
  static constexpr int FM = BM / 2 / 16, FN = BN / 2 / 16;
  static constexpr int NT = 256;
  static constexpr int NVA = BM * BK / 8, NVB = BN * BK / 8;   // 16-byte vectors per tile
  static constexpr int VA = (NVA + NT - 1) / NT;                 // per thread (last guarded)
  static constexpr int VB = (NVB + NT - 1) / NT;
  struct Smem {
    uint16_t a[2][BM][SK];
    uint16_t b[2][BN][SK];
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
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < T::VA; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      if (e < T::NVA) *(uint4*)&sm.a[buf][row][kc] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < T::VB; ++u) {
      int e = tid + u * 256, row = e / (T::BK / 8), kc = (e % (T::BK / 8)) * 8;
      if (e < T::NVB) *(uint4*)&sm.b[buf][row][kc] = rb[u];
    }
  };
  if (K > 0) {
    fetch(0);
    stash(0);
    __syncthreads();
  }
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += T::BK) {
    const bool more = k0 + T::BK < K;
    if (more) fetch(k0 + T::BK);
#pragma unroll
    for (int kk = 0; kk < T::BK; kk += 32) {
      const int kq = kk + (lane >> 4) * 8;
      bf16x8 af[T::FM], bfr[T::FN];
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
        af[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.a[buf][wm * (BM / 2) + i * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int j = 0; j < T::FN; ++j)
        bfr[j] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.b[buf][wn * (BN / 2) + j * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
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

// ------------------------------------------------------------------------------------
// EA update from bf16 activations on bf16 MFMA: F <- rho F + c * Xh^T Xh (Alg. 1 EA lines),
// upper 128 x 128 tiles, 4 waves of 64 x 64.  The contraction runs over the batch rows of
// X, which are strided in memory: each thread loads an 8 (rows) x 8 (columns) block with
// 16-byte row loads and stores the rows unchanged into LDS (row-major stage, 64 rows of
// the tile's column panel); the MFMA operands, which need 8 consecutive rows of one
// column per lane, come from gfx950's transposing LDS read (ds_read_b64_tr_b16: in each
// group of 16 lanes, lanes 4r..4r+3 address row r of a 4 x 16 block and lane j receives
// its column j), two per operand.  Two LDS buffers: one barrier per 64-row step.
//   Loads: sixteen neighbouring lanes cover one 256-byte row segment of a panel, so each
// load instruction touches few cache lines per lane group; full steps use buffer loads
// with the row in the scalar offset and keep two steps in flight in registers.
//   LDS: 288-byte row pitch, so the four 32-byte row pieces of one transposing read land
// on distinct banks; row stores are contiguous 256-byte segments.
//   Order: tiles in 8 x 8 groups, and per XCD one contiguous share of every factor
// (ea_tile, group_locate_xcd8), so the panels of concurrently running tiles meet in L2.
//   Two workgroups share a compute unit; each one's MFMAs fill the other's barrier and
// load waits (one 8-wave workgroup on 256 x 128 pair tiles, which reads a quarter fewer L2
// bytes per flop, measured slower for that reason).
constexpr int EB_BT = kEaBf16Tile, EB_BK = 64, EB_RP = EB_BT + 16;
struct alignas(16) EbSmem {
  union {
    struct {
      uint16_t a[2][EB_BK][EB_RP];
      uint16_t b[2][EB_BK][EB_RP];
    } g;
    float t[EB_BT][EB_BT + 1];
  };
};

typedef short eb_s4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) eb_s4 eb_lds_s4;
// 8 consecutive rows (k0 .. k0+7 for lane group g = lane / 16) of column m0 + lane % 16 of
// a row-major LDS stage, as one MFMA operand: two transposing reads of 4 rows each.
__device__ __forceinline__ bf16x8 eb_tr_frag(const uint16_t (*P)[EB_RP], int k0, int m0, int lane) {
  const int g = lane >> 4, r = (lane >> 2) & 3, q = lane & 3;
  const uint16_t* p = &P[k0 + 8 * g + r][m0 + 4 * q];
  const eb_s4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((eb_lds_s4*)p);
  const eb_s4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((eb_lds_s4*)(p + 4 * EB_RP));
  typedef short s8 __attribute__((ext_vector_type(8)));
  const s8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// Rows [k0, k0+8) x columns [c0, c0+8) of Xh (bf16, ones column appended at d_in when
// ones != 0, zero beyond d and beyond row ke).
__device__ __forceinline__ void eb_load_block(const uint16_t* X, long ldx, int d_in, int d, bool ones, bool vec,
                                              int k0, int ke, int c0, uint4 v[8]) {
  const bool full = vec && (c0 + 8 <= d_in);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = k0 + r;
    v[r] = make_uint4(0, 0, 0, 0);
    if (k >= ke) continue;
    const uint16_t* p = X + (long)k * ldx + c0;
    if (full) {
      v[r] = *(const uint4*)p;
    } else {
      uint16_t t[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = c0 + j;
        t[j] = (c < d_in) ? p[j] : ((ones && c == d_in && c < d) ? (uint16_t)0x3f80 : (uint16_t)0);
      }
      v[r] = make_uint4(t[0] | ((uint32_t)t[1] << 16), t[2] | ((uint32_t)t[3] << 16),
                        t[4] | ((uint32_t)t[5] << 16), t[6] | ((uint32_t)t[7] << 16));
    }
  }
}

// CONV: the rows are the im2col patches of q.cv's NHWC input (the guarded stage path only)
// CONV: 0 plain activations, else the im2col loader form (1: 16-byte, 2: element loads)
template <int CONV = 0>
__device__ __forceinline__ void ea_bf16_tiles_body(const EaTask& q, int bx, int by) {
  __shared__ EbSmem sm;
  const GemmP& p = q.g;
  int I, J;
  ea_tile(bx, q.T, I, J);
  int kb, ke;
  ea_slice(p.K, q.nks, by, EB_BK, kb, ke);
  const bool diag = (I == J);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int d = p.M, d_in = p.ones_col >= 0 ? p.ones_col : d;
  const bool ones = p.ones_col >= 0;
  const uint16_t* X = p.Ab;
  const long ldx = p.lda;
  const bool vec = ((ldx & 7) == 0) && ((((uintptr_t)X) & 15) == 0);
  // loader role: threads 0..127 fill the A panel (columns of block I), 128..255 the B
  // panel; thread (cg, rg) holds rows rg*8 .. rg*8+7 of columns cg*8 .. cg*8+7
  const int op = wave >> 1, tt = tid & 127, cg = tt & 15, rg = tt >> 4;   // op: wave-uniform
  const bool loader = !(diag && op == 1);
  const int c0 = (op ? J : I) * EB_BT + cg * 8;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 v[8];
  constexpr bool conv = CONV != 0;
  // a thread's 8 x 8 block lies inside the activations (no ones column, no padding): its
  // 8 row loads of full 64-row stages go out unguarded
  const bool inner = !conv && vec && (c0 + 8 <= d_in);
  auto fetch = [&](int k0) {
    if constexpr (CONV != 0) {
      im2col_block<CONV>(X, q.cv, ones, k0 + rg * 8, ke, c0, v);
    } else if (inner && k0 + EB_BK <= ke) {
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = gload16(X + (long)(k0 + rg * 8 + r) * ldx + c0);
    } else {
      eb_load_block(X, ldx, d_in, d, ones, vec, k0 + rg * 8, ke, c0, v);
    }
  };
  auto stash = [&](int buf) {
    uint16_t (*dst)[EB_RP] = op ? sm.g.b[buf] : sm.g.a[buf];
#pragma unroll
    for (int r = 0; r < 8; ++r) *(uint4*)&dst[rg * 8 + r][cg * 8] = v[r];
  };
  // the 8 operand reads of one 32-row half h2 of stage buffer buf
  auto read_frags = [&](int buf, int h2, bf16x8 (&af)[2][4], bf16x8 (&bfr)[2][4]) {
    const uint16_t (*A)[EB_RP] = sm.g.a[buf];
    const uint16_t (*B)[EB_RP] = diag ? sm.g.a[buf] : sm.g.b[buf];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[h2][i] = eb_tr_frag(A, h2 * 32, wm * 64 + i * 16, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) bfr[h2][j] = eb_tr_frag(B, h2 * 32, wn * 64 + j * 16, lane);
  };
  auto mfma_one = [&](const bf16x8 (&af)[2][4], const bf16x8 (&bfr)[2][4], int t) {
    const int h2 = t >> 4, i = (t >> 2) & 3, j = t & 3;
    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h2][i], bfr[h2][j], acc[i][j], 0, 0, 0);
  };
  auto mfma_stage = [&](int buf) {
    bf16x8 af[2][4], bfr[2][4];
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      read_frags(buf, h2, af, bfr);
#pragma unroll
      for (int t = 16 * h2; t < 16 * h2 + 16; ++t) mfma_one(af, bfr, t);
    }
  };
  // Both column panels of the tile hold no partial 8-column group (every group lies inside
  // the activations or wholly beyond them), else the tile takes the guarded path.
  auto panel_clean = [&](int P) {
    const int lo = P * EB_BT, hi = lo + EB_BT;
    return (d_in & 7) == 0 || d_in <= lo || d_in >= hi;
  };
  const bool piped = !conv && vec && d_in >= 8 && panel_clean(I) && panel_clean(J) &&
                     (long)(ke - kb) * ldx * 2 < (1L << 31);
  if (piped) {
    // Full 64-row stages, two stages in flight in registers (va, vb) while the MFMAs run
    // on the LDS stage loaded before them.  Every thread issues the same 8 loads per stage
    // and runs the same branch-free code: a thread whose 8 columns lie beyond the
    // activations gets zeros from the buffer range check (its lane offset is past the
    // end of the buffer), and the ones column, which then starts a group of its own
    // (panel_clean), is set in the first transposed column of its thread.
    const int nfull = (ke - kb) / EB_BK;
    const bool in_x = c0 + 8 <= d_in;
    // buffer loads over the block's row slice: one lane offset for every load, the row
    // in the scalar offset; 2^31 is past the range (< 2^31 bytes), so those loads read 0
    const int row_bytes = (int)ldx * 2;
    const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(X + (long)kb * ldx), (short)0, (ke - kb) * row_bytes, 0x00020000);
    const int vo = in_x ? rg * 8 * row_bytes + c0 * 2 : (int)0x80000000u;
    // the ones column, when it starts this thread's (otherwise zero) group: the first
    // half of every row
    const uint32_t o1 = (ones && c0 == d_in && d_in < d) ? 0x3f80u : 0u;
    auto fetch_full = [&](int k0, uint4 (&w)[8]) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const int so = (k0 - kb) * row_bytes;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(xs, vo, so + r * row_bytes, 0);
        w[r] = make_uint4(x.x, x.y, x.z, x.w);
      }
    };
    // Every wave stashes (on a diagonal tile waves 2-3 fill the unused B buffer).
    auto stash_full = [&](const uint4 (&w)[8], int buf) {
      uint16_t (*dst)[EB_RP] = op ? sm.g.b[buf] : sm.g.a[buf];
#pragma unroll
      for (int r = 0; r < 8; ++r) *(uint4*)&dst[rg * 8 + r][cg * 8] = make_uint4(w[r].x | o1, w[r].y, w[r].z, w[r].w);
    };
    // One stage's MFMAs on buffer buf with the next stage (w) stored into buffer buf ^ 1
    // between them, in an order that scheduling fences keep: the first half's 8 operand
    // reads; its 16 MFMAs with the second half's reads behind the 12th (the operands of
    // rows 0-47 of the wave tile are dead by then); the second half's 16 MFMAs with the 8
    // row stores between them (after every read of the stage, which the compiler cannot
    // prove disjoint from them).
    auto stage_stash = [&](int buf, const uint4 (&w)[8]) {
      bf16x8 af[2][4], bfr[2][4];
      read_frags(buf, 0, af, bfr);
      uint16_t (*dst)[EB_RP] = op ? sm.g.b[buf ^ 1] : sm.g.a[buf ^ 1];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        mfma_one(af, bfr, 2 * c);
        mfma_one(af, bfr, 2 * c + 1);
        if (c == 5) {
          __builtin_amdgcn_sched_barrier(0);
          read_frags(buf, 1, af, bfr);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        mfma_one(af, bfr, 16 + 2 * r);
        mfma_one(af, bfr, 16 + 2 * r + 1);
        *(uint4*)&dst[rg * 8 + r][cg * 8] = make_uint4(w[r].x | o1, w[r].y, w[r].z, w[r].w);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // A stage past the last full one re-reads the last full one: the number of loads in
    // flight is then the same on every path, and a stash waits only for its own register
    // set.
    auto stage_k = [&](int st) { return kb + (st < nfull ? st : nfull - 1) * EB_BK; };
    if (nfull > 0) {
      uint4 va[8], vb[8];
      fetch_full(stage_k(0), va);
      fetch_full(stage_k(1), vb);
      stash_full(va, 0);
      __syncthreads();
      fetch_full(stage_k(2), va);
      int s = 0;
      for (; s + 1 < nfull; s += 2) {
        // stage s on buffer 0 while stage s + 1 (vb) goes to buffer 1
        stage_stash(0, vb);
        __syncthreads();
        fetch_full(stage_k(s + 3), vb);
        // stage s + 1 on buffer 1 while stage s + 2 (va) goes to buffer 0; past the last
        // full stage that copy is never read
        stage_stash(1, va);
        __syncthreads();
        fetch_full(stage_k(s + 4), va);
      }
      if (s < nfull) mfma_stage(0);                   // odd count: the last stage is in buffer 0
    }
    const int kt = kb + nfull * EB_BK;
    if (kt < ke) {
      // ragged last stage with guarded loads; buffer nfull & 1 was last read two stages
      // back, before a barrier
      if (loader) {
        eb_load_block(X, ldx, d_in, d, ones, vec, kt + rg * 8, ke, c0, v);
        stash(nfull & 1);
      }
      __syncthreads();
      mfma_stage(nfull & 1);
    }
  } else {
    if (kb < ke) {
      if (loader) {
        fetch(kb);
        stash(0);
      }
      __syncthreads();
    }
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += EB_BK) {
      const bool more = k0 + EB_BK < ke;
      if (more && loader) fetch(k0 + EB_BK);
      mfma_stage(buf);
      __builtin_amdgcn_sched_barrier(0);             // the stash (and its load waits) after the MFMAs
      if (more && loader) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  auto for_each = [&](auto&& fn) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          fn(wm * 64 + i * 16 + 4 * (lane >> 4) + r, wn * 64 + j * 16 + (lane & 15), acc[i][j][r]);
  };
  if (q.nks > 1) {
    float* slot = p.part + ((long)bx * q.nks + by) * (EB_BT * EB_BT);
    for_each([&](int r, int c, float x) { slot[r * EB_BT + c] = x; });
    return;
  }
  __syncthreads();
  for_each([&](int r, int c, float x) { sm.t[r][c] = x; });
  __syncthreads();
  ea_store_tile_t<EB_BT>(sm.t, q.o, I, J);
}

__device__ __forceinline__ void ea_bf16_finalize_body(const EaTask& q, int bx, int) {
  __shared__ float v[kEaChunk][EB_BT + 1];
  ea_finalize_chunk<EB_BT>(q, bx, v);
}

// Patch staging (conv_patch_bytes): thread t writes rows 8 (t / G) .. +7 of column group
// t % G (G = ldp / 8) of P, gathered with the im2col loader's 16-byte form (FORM 1, g.vec)
// or its element form (FORM 2).
template <int FORM>
__global__ __launch_bounds__(256) void k_im2col_stage(const uint16_t* x, ConvGeom g, uint16_t* P, int ldp, int n) {
  const int groups = ldp / 8;
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long rb = t / groups;
  const int cgp = (int)(t - rb * groups);
  const long k0 = rb * 8;
  if (k0 >= n) return;
  uint4 v[8];
  im2col_block<FORM>(x, g, false, (int)k0, n, cgp * 8, v);
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (k0 + r < n) *(uint4*)&P[(k0 + r) * ldp + cgp * 8] = v[r];
}
hipError_t launch_im2col_stage(const uint16_t* x, const ConvGeom& g, uint16_t* P, int ldp, int n, hipStream_t s) {
  const long threads = (long)((n + 7) / 8) * (ldp / 8);
  const dim3 grid((unsigned)((threads + 255) / 256));
  if (threads > 0 && g.vec) hipLaunchKernelGGL(k_im2col_stage<1>, grid, dim3(256), 0, s, x, g, P, ldp, n);
  else if (threads > 0) hipLaunchKernelGGL(k_im2col_stage<2>, grid, dim3(256), 0, s, x, g, P, ldp, n);
  return hipGetLastError();
}

// blocks spread over the XCDs so that consecutive tiles of one slice share an L2
__global__ __launch_bounds__(256) void k_ea_bf16_tiles(EaTask q) {
  const int l = xcd_swizzle(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  ea_bf16_tiles_body(q, l % gridDim.x, l / gridDim.x);
}
template <int FORM>
__global__ __launch_bounds__(256) void k_ea_bf16_tiles_conv(EaTask q) {
  const int l = xcd_swizzle(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  ea_bf16_tiles_body<FORM>(q, l % gridDim.x, l / gridDim.x);
}
__global__ __launch_bounds__(256) void k_ea_bf16_finalize(EaTask q) { ea_bf16_finalize_body(q, blockIdx.x, 0); }
// grouped EA tiles: per-task block counts padded to multiples of 8 (the padding blocks
// have slice index >= nks and exit)
__global__ __launch_bounds__(256) void k_ea_bf16_tiles_g(const EaTask* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate_xcd8(gm, t, bx, by);
  if (by >= tasks[t].nks) return;
  ea_bf16_tiles_body(tasks[t], bx, by);
}
KFAC_GROUPED_KERNEL(k_ea_bf16_finalize_g, ea_bf16_finalize_body, EaTask, 256)

hipError_t launch_ea_bf16_tiles(const EaTask& q, int tiles, int ks, hipStream_t s) {
  if (q.cv.C > 0 && q.cv.vec) hipLaunchKernelGGL(k_ea_bf16_tiles_conv<1>, dim3(tiles, ks), dim3(256), 0, s, q);
  else if (q.cv.C > 0) hipLaunchKernelGGL(k_ea_bf16_tiles_conv<2>, dim3(tiles, ks), dim3(256), 0, s, q);
  else hipLaunchKernelGGL(k_ea_bf16_tiles, dim3(tiles, ks), dim3(256), 0, s, q);
  return hipGetLastError();
}
hipError_t launch_ea_bf16_finalize(const EaTask& q, int tiles, hipStream_t s) {
  hipLaunchKernelGGL(k_ea_bf16_finalize, dim3(tiles * ea_finalize_chunks(true)), dim3(256), 0, s, q);
  return hipGetLastError();
}
hipError_t launch_ea_bf16_tiles_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_ea_bf16_tiles_g, dim3(blocks), dim3(256), 0, s, t, gm);
  return hipGetLastError();
}
hipError_t launch_ea_bf16_finalize_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_ea_bf16_finalize_g, dim3(blocks), dim3(256), 0, s, t, gm);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
constexpr int BF_BM = 96, BF_BN = 128;
__global__ __launch_bounds__(256) void k_gemm_bf16_nt(BfGemmTask q) { gemm_bf16_body<BF_BM, BF_BN>(q, blockIdx.x, 0); }
__global__ __launch_bounds__(256) void k_gemm_bf16_nt_g(const BfGemmTask* tasks, GroupMap gm) {
  int t, bx, by;
  group_locate_xcd(gm, t, bx, by);
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
// ------------------------------------------------------------------------------------
// Skinny sketch GEMM for the range finder (Alg. 3 "compute X Omega" and the power
// iterations): C[M x N] = A[M x K] B[N x K]^T with M = l_pad <= 288 (the sketch width)
// and N = K = d large.  A workgroup owns all M rows and 256 columns of C over one K slice,
// so every element of F (B) is read once per slice and each 32-deep step issues 36 MFMAs
// per wavefront for 13 LDS operand reads.  8 wavefronts as 2 (M) x 4 (N), each 144 x 64
// (9 x 4 tiles of 16 x 16); BK = 64 with two LDS buffers.  K slices write fp32 partials
// that a second launch sums in slice order.
constexpr int SK_BN = 256, SK_MMAX = 288, SK_BK = 64, SK_SK = SK_BK + 8, SK_NT = 512;
struct alignas(16) SkSmem {
  uint16_t a[2][SK_MMAX][SK_SK];
  uint16_t b[2][SK_BN][SK_SK];
};
constexpr int SK_VA = (SK_MMAX * SK_BK / 8 + SK_NT - 1) / SK_NT;   // 16-byte vectors per thread
constexpr int SK_VB = SK_BN * SK_BK / 8 / SK_NT;

__device__ __forceinline__ void skinny_body(const SkinnyTask& task, int bx, int by) {
  __shared__ SkSmem sm;
  const SkinnyTask q = task;                         // the record once, into registers
  const int tn = bx, ks = by;                        // grid width = tiles_n
  const int n0 = tn * SK_BN;
  const int M = q.M, N = q.N, K = q.K;
  const int kchunk = ((K + q.ksplit - 1) / q.ksplit + SK_BK - 1) / SK_BK * SK_BK;
  const int kb = ks * kchunk, ke = min(K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int mt = (M + 15) / 16;                      // m tiles present
  f32x4 acc[9][4];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ra[SK_VA], rb[SK_VB];
  uint32_t ma[SK_VA], mb[SK_VB];                     // applied at the stash, not at the load
  // Full stages of 16-byte aligned rows load without element guards: a row outside the
  // matrix reads a clamped valid address and is zeroed through the mask at the stash, so
  // the loads stay in flight across the MFMAs.  The K tail and unaligned operands take the
  // guarded ld16 in an unpipelined loop after the main one.
  const bool al = (((q.lda | q.ldb) & 7) == 0) && (((uintptr_t)q.A | (uintptr_t)q.B) & 15) == 0;
  const int kfull = al ? kb + (ke - kb) / SK_BK * SK_BK : kb;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SK_VA; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      const bool ok = e < SK_MMAX * SK_BK / 8 && row < M;
      ra[u] = gload16(q.A + (ok ? (long)row * q.lda + k0 + kc : 0));
      ma[u] = opaque_mask(ok);
    }
#pragma unroll
    for (int u = 0; u < SK_VB; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      const bool ok = n0 + row < N;
      rb[u] = gload16(q.B + (ok ? (long)(n0 + row) * q.ldb + k0 + kc : 0));
      mb[u] = opaque_mask(ok);
    }
  };
  auto fetch_guarded = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SK_VA; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      ra[u] = (e < SK_MMAX * SK_BK / 8 && row < M) ? ld16(q.A, q.lda, row, M, k0 + kc, ke) : make_uint4(0, 0, 0, 0);
      ma[u] = 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < SK_VB; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      rb[u] = ld16(q.B, q.ldb, n0 + row, N, k0 + kc, ke);
      mb[u] = 0xffffffffu;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < SK_VA; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      if (e < SK_MMAX * SK_BK / 8) *(uint4*)&sm.a[buf][row][kc] = and_mask(ra[u], ma[u]);
    }
#pragma unroll
    for (int u = 0; u < SK_VB; ++u) {
      const int e = tid + u * SK_NT, row = e >> 3, kc = (e & 7) * 8;
      *(uint4*)&sm.b[buf][row][kc] = and_mask(rb[u], mb[u]);
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < SK_BK; kk += 32) {
      const int kq = kk + (lane >> 4) * 8;
      bf16x8 bfr[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bfr[j] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.b[buf][wn * 64 + j * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if (wm * 9 + i < mt) {                        // uniform: skip m tiles beyond M
          const bf16x8 af = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.a[buf][wm * 144 + i * 16 + (lane & 15)][kq]);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[j], acc[i][j], 0, 0, 0);
        }
      }
    }
  };
  int buf = 0;
  if (kb < kfull) {
    fetch(kb);
    stash(0);
    __syncthreads();
  }
  for (int k0 = kb; k0 < kfull; k0 += SK_BK) {
    // the last full stage re-fetches itself into the idle buffer (never read)
    fetch(k0 + SK_BK < kfull ? k0 + SK_BK : k0);
    compute(buf);
    __builtin_amdgcn_sched_barrier(0);               // keep the stash (and its load waits) after the MFMAs
    stash(buf ^ 1);                                   // its last reads closed at the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  for (int k0 = kfull; k0 < ke; k0 += SK_BK) {
    fetch_guarded(k0);
    stash(buf);
    __syncthreads();
    compute(buf);
    __syncthreads();
  }
  const long ldp = (N + 3) / 4 * 4;                 // partial row pitch (16-byte rows)
  float* out = (q.ksplit > 1) ? q.part + (long)ks * M * ldp : q.C;
  const long ldo = (q.ksplit > 1) ? ldp : q.ldc;
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 144 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < M && col < N) out[(long)row * ldo + col] = acc[i][j][r];
      }
}

// ------------------------------------------------------------------------------------
// The Rayleigh-Ritz product W = F Q (Alg. 3 "C = Q^T X Q") in the bf16-sketch precision
// mode.  fp32 has 1/16 of bf16's MFMA rate on gfx950, so each fp32 operand enters as a
// pair of bf16 values, hi = bf16(v) and lo = bf16(v - hi) (v - hi is exact in fp32), and
// C = A_hi B_hi + A_hi B_lo + A_lo B_hi accumulates in fp32: each product keeps 16
// significant bits per operand and drops only lo*lo (below 2^-16 relative).  The split is
// done once per element while staging into LDS.  Same whole-width layout as the sketch
// kernel: a workgroup owns all M <= 288 rows and 128 columns of C over one K slice, so F is
// read from memory once; 8 wavefronts as 2 (M) x 4 (N), each 144 x 32 (9 x 2 tiles); BK =
// 32 with two LDS buffers of hi and lo planes (130 KB).  K slices write fp32 partials.
constexpr int SS_BN = 128, SS_BK = 32, SS_SK = SS_BK + 8, SS_NT = 512;
struct alignas(16) SsSmem {
  uint16_t ah[2][SK_MMAX][SS_SK], al[2][SK_MMAX][SS_SK];
  uint16_t bh[2][SS_BN][SS_SK], bl[2][SS_BN][SS_SK];
};
constexpr int SS_NVA = SK_MMAX * SS_BK / 4, SS_NVB = SS_BN * SS_BK / 4;     // float4 per stage
constexpr int SS_VA = (SS_NVA + SS_NT - 1) / SS_NT, SS_VB = SS_NVB / SS_NT;  // per thread
static_assert(SS_NVB % SS_NT == 0, "B stage must divide evenly");

// 4 consecutive fp32 of row `row` from column k (zeros outside rows < nrows, k < K).
__device__ __forceinline__ float4 ld4f(const float* base, long ld, int row, int nrows, int k, int K) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row < nrows) {
    const float* p = base + (long)row * ld + k;
    if (k + 4 <= K && (((uintptr_t)p) & 15) == 0) {
      v = *(const float4*)p;
    } else {
      v.x = (k < K) ? p[0] : 0.f;
      v.y = (k + 1 < K) ? p[1] : 0.f;
      v.z = (k + 2 < K) ? p[2] : 0.f;
      v.w = (k + 3 < K) ? p[3] : 0.f;
    }
  }
  return v;
}

// hi / lo bf16 planes of 4 values, stored as one 8-byte word each (v - hi is exact in fp32)
__device__ __forceinline__ void split_store(const float4 v, uint16_t* hi, uint16_t* lo) {
  const uint32_t h0 = pack_bf16x2(v.x, v.y), h1 = pack_bf16x2(v.z, v.w);
  const uint32_t l0 = pack_bf16x2(v.x - __uint_as_float(h0 << 16), v.y - __uint_as_float(h0 & 0xffff0000u));
  const uint32_t l1 = pack_bf16x2(v.z - __uint_as_float(h1 << 16), v.w - __uint_as_float(h1 & 0xffff0000u));
  *(uint2*)hi = make_uint2(h0, h1);
  *(uint2*)lo = make_uint2(l0, l1);
}

template <bool AL>
__device__ __forceinline__ void split_run(const SplitTask& q, SsSmem& sm, int bx, int by) {
  const int tn = bx, ks = by;                        // grid width = tiles_n
  const int n0 = tn * SS_BN;
  const int M = q.M, N = q.N, K = q.K;
  const int kchunk = ((K + q.ksplit - 1) / q.ksplit + SS_BK - 1) / SS_BK * SS_BK;
  const int kb = ks * kchunk, ke = min(K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int mt = (M + 15) / 16;                      // m tiles present
  f32x4 acc[9][2];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ra[SS_VA], rb[SS_VB];                        // fp32 bits
  uint32_t ma[SS_VA], mb[SS_VB];                     // applied at the stash, not at the load
  // Full stages load without element guards: a row outside the matrix reads a clamped valid
  // address and is zeroed through the mask at the stash, so the loads stay in flight across
  // the MFMAs.  AL: 16-byte aligned rows (one 16-byte load per 4 values), else four 4-byte
  // loads.  The K tail takes the guarded ld4f in an unpipelined loop after the main one.
  const int kfull = kb + (ke - kb) / SS_BK * SS_BK;
  auto ld_full = [&](const float* p) -> uint4 {
    if constexpr (AL) {
      return gload16(p);
    } else {
      return make_uint4(gload4(p), gload4(p + 1), gload4(p + 2), gload4(p + 3));
    }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SS_VA; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      const bool ok = e < SS_NVA && row < M;
      ra[u] = ld_full(q.A + (ok ? (long)row * q.lda + k0 + kc : 0));
      ma[u] = opaque_mask(ok);
    }
#pragma unroll
    for (int u = 0; u < SS_VB; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      const bool ok = n0 + row < N;
      rb[u] = ld_full(q.B + (ok ? (long)(n0 + row) * q.ldb + k0 + kc : 0));
      mb[u] = opaque_mask(ok);
    }
  };
  auto fetch_guarded = [&](int k0) {
#pragma unroll
    for (int u = 0; u < SS_VA; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      ra[u] = __builtin_bit_cast(uint4, (e < SS_NVA) ? ld4f(q.A, q.lda, row, M, k0 + kc, ke)
                                                      : make_float4(0.f, 0.f, 0.f, 0.f));
      ma[u] = 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < SS_VB; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      rb[u] = __builtin_bit_cast(uint4, ld4f(q.B, q.ldb, n0 + row, N, k0 + kc, ke));
      mb[u] = 0xffffffffu;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < SS_VA; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      if (e < SS_NVA)
        split_store(__builtin_bit_cast(float4, and_mask(ra[u], ma[u])), &sm.ah[buf][row][kc], &sm.al[buf][row][kc]);
    }
#pragma unroll
    for (int u = 0; u < SS_VB; ++u) {
      const int e = tid + u * SS_NT, row = e >> 3, kc = (e & 7) * 4;
      split_store(__builtin_bit_cast(float4, and_mask(rb[u], mb[u])), &sm.bh[buf][row][kc], &sm.bl[buf][row][kc]);
    }
  };
  const int kq = (lane >> 4) * 8;
  auto compute = [&](int buf) {
    bf16x8 bh[2], bl[2], ah[9], al[9];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = wn * 32 + j * 16 + (lane & 15);
      bh[j] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.bh[buf][row][kq]);
      bl[j] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.bl[buf][row][kq]);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int row = wm * 144 + i * 16 + (lane & 15);
      ah[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.ah[buf][row][kq]);
      al[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&sm.al[buf][row][kq]);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
      if (wm * 9 + i < mt)                           // uniform: skip m tiles beyond M
#pragma unroll
        for (int j = 0; j < 2; ++j) {                // small terms first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
  };
  int buf = 0;
  if (kb < kfull) {
    fetch(kb);
    stash(0);
    __syncthreads();
  }
  for (int k0 = kb; k0 < kfull; k0 += SS_BK) {
    // the last full stage re-fetches itself into the idle buffer (never read)
    fetch(k0 + SS_BK < kfull ? k0 + SS_BK : k0);
    compute(buf);
    __builtin_amdgcn_sched_barrier(0);               // keep the stash (and its load waits) after the MFMAs
    stash(buf ^ 1);                                   // its last reads closed at the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  for (int k0 = kfull; k0 < ke; k0 += SS_BK) {
    fetch_guarded(k0);
    stash(buf);
    __syncthreads();
    compute(buf);
    __syncthreads();
  }
  const long ldp = (N + 3) / 4 * 4;                 // partial row pitch (16-byte rows)
  float* out = (q.ksplit > 1) ? q.part + (long)ks * M * ldp : q.C;
  const long ldo = (q.ksplit > 1) ? ldp : q.ldc;
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 144 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) out[(long)row * ldo + col] = acc[i][j][r];
      }
}

__device__ __forceinline__ void split_body(const SplitTask& task, int bx, int by) {
  __shared__ SsSmem sm;
  const SplitTask q = task;                          // the record once, into registers
  if ((((q.lda | q.ldb) & 3) == 0) && (((uintptr_t)q.A | (uintptr_t)q.B) & 15) == 0)
    split_run<true>(q, sm, bx, by);
  else
    split_run<false>(q, sm, bx, by);
}

// Sum of the K-slice partials, in slice order: block = 256 threads x 4 consecutive columns
// of one row (16-byte loads of the partials; the partial row pitch is a multiple of 4).
__device__ __forceinline__ void reduce_body(const ReduceTask& q, int bx, int) {
  const int N4 = (q.N + 3) / 4;
  const long ldp = (long)N4 * 4;
  const long total = (long)q.M * ldp;
  const long g = (long)bx * 256 + threadIdx.x;       // group of 4 columns
  if (g >= (long)q.M * N4) return;
  const int row = (int)(g / N4), col = (int)(g % N4) * 4;
  const float* p = q.part + (long)row * ldp + col;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = 0; k < q.ksplit; ++k) {             // pad columns >= N are summed, never stored
    const float4 v = *(const float4*)(p + (long)k * total);
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  float* c = q.C + (long)row * q.ldc + col;
  c[0] = s.x;
  if (col + 1 < q.N) c[1] = s.y;
  if (col + 2 < q.N) c[2] = s.z;
  if (col + 3 < q.N) c[3] = s.w;
}

__global__ __launch_bounds__(SK_NT) void k_skinny_bf16(SkinnyTask q) { skinny_body(q, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(SS_NT) void k_split_bf16x3(SplitTask q) { split_body(q, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(256) void k_slice_reduce(ReduceTask q) { reduce_body(q, blockIdx.x, 0); }
KFAC_GROUPED_KERNEL_XCD(k_skinny_bf16_g, skinny_body, SkinnyTask, SK_NT)
KFAC_GROUPED_KERNEL_XCD(k_split_bf16x3_g, split_body, SplitTask, SS_NT)
KFAC_GROUPED_KERNEL(k_slice_reduce_g, reduce_body, ReduceTask, 256)

// K slices for a whole-width kernel with `tiles` column tiles: about one workgroup per
// compute unit, at least 512 k per slice, at most 16 slices.
static int ksplit_for(int tiles, int K) {
  int ks = (256 + tiles - 1) / tiles;
  ks = std::min(ks, std::max(1, K / 512));
  return std::max(1, std::min(ks, 16));
}
int skinny_ksplit(int N, int K) { return ksplit_for((N + SK_BN - 1) / SK_BN, K); }
int split_ksplit(int N, int K) { return ksplit_for((N + SS_BN - 1) / SS_BN, K); }
SkinnyTask make_skinny_task(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb, float* C,
                            long ldc, float* part, int ksplit) {
  SkinnyTask q{M, N, K, A, lda, B, ldb, C, ldc, part, ksplit, (N + SK_BN - 1) / SK_BN};
  return q;
}
SplitTask make_split_task(int M, int N, int K, const float* A, long lda, const float* B, long ldb, float* C,
                          long ldc, float* part, int ksplit) {
  SplitTask q{M, N, K, A, lda, B, ldb, C, ldc, part, ksplit, (N + SS_BN - 1) / SS_BN};
  return q;
}
ReduceTask make_reduce_task(int M, int N, const float* part, float* C, long ldc, int ksplit) {
  ReduceTask q{M, N, part, C, ldc, ksplit};
  return q;
}
int skinny_blocks(const SkinnyTask& q) { return q.tiles_n * q.ksplit; }
int split_blocks(const SplitTask& q) { return q.tiles_n * q.ksplit; }
int reduce_blocks(const ReduceTask& q) { return (int)(((long)q.M * ((q.N + 3) / 4) + 255) / 256); }
static size_t part_bytes(int M, int N, int ks) {
  return ks > 1 ? (size_t)ks * M * ((N + 3) / 4 * 4) * sizeof(float) : 0;
}
size_t skinny_part_bytes(int M, int N, int K) { return part_bytes(M, N, skinny_ksplit(N, K)); }
size_t split_part_bytes(int M, int N, int K) { return part_bytes(M, N, split_ksplit(N, K)); }
hipError_t launch_skinny_g(const SkinnyTask* t, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_skinny_bf16_g, dim3(blocks), dim3(SK_NT), 0, s, t, gm);
  return hipGetLastError();
}
hipError_t launch_split_g(const SplitTask* t, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_split_bf16x3_g, dim3(blocks), dim3(SS_NT), 0, s, t, gm);
  return hipGetLastError();
}
hipError_t launch_skinny(const SkinnyTask& q, hipStream_t s) {
  if (q.M > SK_MMAX) return hipErrorInvalidValue;
  if (q.M <= 0 || q.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_skinny_bf16, dim3(q.tiles_n, q.ksplit), dim3(SK_NT), 0, s, q);
  if (q.ksplit > 1) {
    const ReduceTask r = make_reduce_task(q.M, q.N, q.part, q.C, q.ldc, q.ksplit);
    hipLaunchKernelGGL(k_slice_reduce, dim3(reduce_blocks(r)), dim3(256), 0, s, r);
  }
  return hipGetLastError();
}
hipError_t launch_split(const SplitTask& q, hipStream_t s) {
  if (q.M > SK_MMAX) return hipErrorInvalidValue;
  if (q.M <= 0 || q.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_bf16x3, dim3(q.tiles_n, q.ksplit), dim3(SS_NT), 0, s, q);
  if (q.ksplit > 1) {
    const ReduceTask r = make_reduce_task(q.M, q.N, q.part, q.C, q.ldc, q.ksplit);
    hipLaunchKernelGGL(k_slice_reduce, dim3(reduce_blocks(r)), dim3(256), 0, s, r);
  }
  return hipGetLastError();
}
hipError_t launch_reduce_g(const ReduceTask* t, GroupMap gm, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_slice_reduce_g, dim3(blocks), dim3(256), 0, s, t, gm);
  return hipGetLastError();
}

}  // namespace kfac
