// Epilogue shared by the fp32- and bf16-operand EA kernels: blend one BT x BT tile of
// raw sums into the factor (F <- rho F + c * sums, Alg. 1's EA lines) and write the
// tile and its mirror, plus the optional bf16 shadow of F.
#pragma once
#include "tasks.h"
#include "gemm_f32.h"

namespace kfac {

// (I, J) of the t-th upper tile of an EA factor with T tiles per side, in groups of
// 8 x 8 tiles (row-major over the upper groups, row-major inside a group).  Consecutive
// tiles, which run together on one XCD, then read 16 column panels of the activations
// (8 on the diagonal) instead of a whole tile row's worth, and share them through that
// XCD's L2.  Producers and the split-K finalize use the same order.
__device__ __forceinline__ void ea_tile(int t, int T, int& I, int& J) {
  constexpr int G = 8;
  const int NG = (T + G - 1) / G;
  int P = 0, Q = 0, rem = t;
  for (;;) {
    const int nr = min(G, T - P * G), nc = min(G, T - Q * G);
    const int cnt = (P == Q) ? nr * (nr + 1) / 2 : nr * nc;
    if (rem < cnt) {
      if (P == Q) {
        int i = 0;
        while (rem >= nr - i) { rem -= nr - i; ++i; }
        I = P * G + i; J = P * G + i + rem;
      } else {
        I = P * G + rem / nc; J = Q * G + rem % nc;
      }
      return;
    }
    rem -= cnt;
    if (++Q == NG) { ++P; Q = P; }
  }
}

// `t` holds the raw sums of upper tile (I, J) (rows of block I, columns of block J); the
// workgroup has NT threads.  The old upper-block values of F are loaded in batches of 16
// per thread before any of them is used, so that each wave keeps 16 loads in flight: a
// load-use loop would leave one load per wave in flight and make this epilogue, not the
// products, the cost of tiles with short contractions.  Each element is read, blended and
// stored by one thread; on a diagonal tile only the upper triangle is read and stored, and
// the mirror pass writes the lower one from the blended upper values (exact symmetry).
template <int BT, int NT = 256>
__device__ __forceinline__ void ea_store_tile_t(float (*t)[BT + 1], const EaOut& o, int I, int J) {
  constexpr int PER = BT * BT / NT, BATCH = PER < 16 ? PER : 16, RS = NT / BT;
  static_assert(NT % BT == 0 && PER % BATCH == 0, "tile / workgroup shape");
  // thread tid handles rows a0 + RS u (u < PER) of column b of the tile
  const int tid = threadIdx.x, a0 = tid / BT, b = tid % BT;
  const int r0 = I * BT, c0 = J * BT;
  const bool dg = (I == J);
  const long step = (long)RS * o.ldf, stepb = (long)RS * o.ldfb;
  // upper block (rows of I, columns of J), coalesced along columns
  {
    float* const src = o.F + (long)(r0 + a0) * o.ldf + (c0 + b);
    uint16_t* const srcb = o.Fb ? o.Fb + (long)(r0 + a0) * o.ldfb + (c0 + b) : nullptr;
    const bool colok = c0 + b < o.d;
#pragma unroll
    for (int u0 = 0; u0 < PER; u0 += BATCH) {
      float f[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int a = a0 + RS * (u0 + u);
        f[u] = (colok && r0 + a < o.d && (!dg || a <= b)) ? src[(u0 + u) * step] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int a = a0 + RS * (u0 + u);
        const bool st = colok && r0 + a < o.d && (!dg || a <= b);
        const float v = st ? o.rho * f[u] + o.c * t[a][b] : 0.f;
        t[a][b] = v;
        if (st) {
          src[(u0 + u) * step] = v;
          if (srcb) srcb[(u0 + u) * stepb] = f32_to_bf16_rne(v);
        }
      }
    }
  }
  __syncthreads();
  // mirror block (rows of J, columns of I): element (c0 + a, r0 + b) = t[b][a]
  {
    float* const dst = o.F + (long)(c0 + a0) * o.ldf + (r0 + b);
    uint16_t* const dstb = o.Fb ? o.Fb + (long)(c0 + a0) * o.ldfb + (r0 + b) : nullptr;
    const bool colok = r0 + b < o.d;
#pragma unroll 8
    for (int u = 0; u < PER; ++u) {
      const int a = a0 + RS * u;
      if (colok && c0 + a < o.d && (!dg || b < a)) {
        const float v = t[b][a];
        dst[u * step] = v;
        if (dstb) dstb[u * stepb] = f32_to_bf16_rne(v);
      }
    }
  }
}

// Deterministic split-K reduction of tile bx (slices summed in index order) into t.
template <int BT>
__device__ void ea_sum_slices(float (*t)[BT + 1], const float* base, int nks) {
  for (int e = threadIdx.x; e < BT * BT; e += blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < nks; ++k) s += base[(long)k * BT * BT + e];
    t[e / BT][e % BT] = s;
  }
}

// Split-K finalize of one 16-row chunk of an upper BT x BT tile: block bx = tile * (BT/16)
// + chunk.  Sums the slices in index order, blends into F (upper element read once, the
// blended value written to the element and its mirror) and refreshes the bf16 shadow.
constexpr int kEaChunk = 16;
template <int BT>
__device__ void ea_finalize_chunk(const EaTask& q, int bx, float (*v)[BT + 1]) {
  constexpr int NCH = BT / kEaChunk;
  const int tile = bx / NCH, a0 = (bx % NCH) * kEaChunk;
  int I, J;
  ea_tile(tile, q.T, I, J);
  const EaOut& o = q.o;
  const int r0 = I * BT, c0 = J * BT, nks = q.nks;
  const float* base = q.g.part + (long)tile * nks * (BT * BT) + (long)a0 * BT;
  for (int e = threadIdx.x; e < kEaChunk * BT; e += blockDim.x) {
    float s = 0.f;
#pragma unroll 8
    for (int k = 0; k < nks; ++k) s += base[(long)k * BT * BT + e];
    const int a = e / BT, b = e % BT;
    const int i = r0 + a0 + a, j = c0 + b;
    float val = 0.f;
    if (i < o.d && j < o.d) {
      val = o.rho * o.F[(long)i * o.ldf + j] + o.c * s;
      if (I != J || a0 + a <= b) {
        o.F[(long)i * o.ldf + j] = val;
        if (o.Fb) o.Fb[(long)i * o.ldfb + j] = f32_to_bf16_rne(val);
      }
    }
    v[a][b] = val;
  }
  __syncthreads();
  // mirror: element (c0 + b, r0 + a0 + a) = v[a][b], 16 contiguous columns per row
  for (int e = threadIdx.x; e < kEaChunk * BT; e += blockDim.x) {
    const int b = e / kEaChunk, a = e % kEaChunk;
    const int i = c0 + b, j = r0 + a0 + a;
    if (i < o.d && j < o.d && (I != J || b > a0 + a)) {
      const float val = v[a][b];
      o.F[(long)i * o.ldf + j] = val;
      if (o.Fb) o.Fb[(long)i * o.ldfb + j] = f32_to_bf16_rne(val);
    }
  }
}

// K range [kb, ke) of slice ks out of nks over K rows, in multiples of bk.
__device__ __forceinline__ void ea_slice(int K, int nks, int ks, int bk, int& kb, int& ke) {
  const int kchunk = ((K + nks - 1) / nks + bk - 1) / bk * bk;
  kb = ks * kchunk;
  ke = min(K, kb + kchunk);
}

}  // namespace kfac
