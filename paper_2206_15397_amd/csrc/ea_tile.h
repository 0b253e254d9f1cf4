// Epilogue shared by the fp32- and bf16-operand EA kernels: blend one BT x BT tile of
// raw sums into the factor (F <- rho F + c * sums, Alg. 1's EA lines) and write the
// tile and its mirror, plus the optional bf16 shadow of F.
#pragma once
#include "tasks.h"

namespace kfac {

// `t` holds the raw sums of upper tile (I, J) (rows of block I, columns of block J).
template <int BT>
__device__ void ea_store_tile_t(float (*t)[BT + 1], const EaOut& o, int I, int J) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r0 = I * BT, c0 = J * BT;
  // upper block (rows of I, columns of J), coalesced along columns
  for (int e = tid; e < BT * BT; e += nt) {
    const int a = e / BT, b = e % BT;
    const int i = r0 + a, j = c0 + b;
    float v = 0.f;
    if (i < o.d && j < o.d) v = o.rho * o.F[(long)i * o.ldf + j] + o.c * t[a][b];
    t[a][b] = v;   // same thread reads and writes the same slot
  }
  __syncthreads();
  for (int e = tid; e < BT * BT; e += nt) {
    const int a = e / BT, b = e % BT;
    const int i = r0 + a, j = c0 + b;
    if (i < o.d && j < o.d && (I != J || a <= b)) {
      const float v = t[a][b];
      o.F[(long)i * o.ldf + j] = v;
      if (o.Fb) o.Fb[(long)i * o.ldfb + j] = f32_to_bf16_rne(v);
    }
  }
  // mirror block (rows of J, columns of I): element (c0+a, r0+b) = t[b][a]
  for (int e = tid; e < BT * BT; e += nt) {
    const int a = e / BT, b = e % BT;
    const int i = c0 + a, j = r0 + b;
    if (i < o.d && j < o.d && (I != J || b < a)) {
      const float v = t[b][a];
      o.F[(long)i * o.ldf + j] = v;
      if (o.Fb) o.Fb[(long)i * o.ldfb + j] = f32_to_bf16_rne(v);
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

// K range [kb, ke) of slice ks out of nks over K rows, in multiples of bk.
__device__ __forceinline__ void ea_slice(int K, int nks, int ks, int bk, int& kb, int& ke) {
  const int kchunk = ((K + nks - 1) / nks + bk - 1) / bk * bk;
  kb = ks * kchunk;
  ke = min(K, kb + kchunk);
}

}  // namespace kfac
