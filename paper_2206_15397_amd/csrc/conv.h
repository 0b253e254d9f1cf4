// im2col addressing of a convolution's patch matrix (ConvGeom in tasks.h), read straight
// from the NHWC input by the loaders of the EA and weight-gradient kernels: the patches
// are never materialised.
#pragma once
#include "tasks.h"

namespace kfac {

__host__ __device__ inline int conv_out(int in, int k, int pad, int stride) { return (in + 2 * pad - k) / stride + 1; }

// Rows [k0, k0+8) x columns [c0, c0+8) of [P | 1] (P: the im2col patches, n = B Ho Wo rows,
// kh kw C columns; the ones column at index kh kw C when `ones`), zero beyond row K.
// Eight columns of one tap are eight consecutive channels of one input pixel: one 16-byte
// load when g.vec (C a multiple of 8, x 16-byte aligned), element loads otherwise.  The
// output position (b, oh, ow) of row k0 and the tap (dy, dx, c) of column c0 take four
// divisions per call, each a multiply and shift by the geometry's precomputed reciprocals
// (an integer division expands to about 25 instructions in this VALU-bound loader); the
// later rows and columns step from them (a row advances ow, wrapping into oh and b; a
// column advances c, wrapping into dx and dy).
//   FORM 0 chooses per call from g.vec; FORM 1 is the 16-byte form only (g.vec set: C and so
// kh kw C are multiples of 8, so a column group lies wholly inside the patch or wholly
// past it, where only the ones column is nonzero); FORM 2 the element form only.  A
// kernel built for one form does not carry the other's code (a shared body measured
// 5-8% slower on the 16-byte layers).
template <int FORM = 0>
__device__ __forceinline__ void im2col_block(const uint16_t* x, const ConvGeom& g, bool ones, int k0, int K, int c0,
                                             uint4 v[8]) {
  const int ncols = g.kh * g.kw * g.C;
  const int howo = g.Ho * g.Wo;
  if (FORM == 1 && c0 >= ncols) {
    const uint32_t o1 = (ones && c0 == ncols) ? 0x3f80u : 0u;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = make_uint4(k0 + r < K ? o1 : 0u, 0u, 0u, 0u);
    return;
  }
  const bool vec8 = FORM == 1 || (FORM == 0 && g.vec && c0 + 8 <= ncols);
  const int cc = c0 < ncols ? c0 : 0;
  const int tap0 = conv_div(cc, g.dC), ch0 = cc - tap0 * g.C, dy0 = conv_div(tap0, g.dKw), dx0 = tap0 - dy0 * g.kw;
  const int kk = k0 < K ? k0 : 0;
  int b = conv_div(kk, g.dHoWo);
  const int rem = kk - b * howo;
  int oh = conv_div(rem, g.dWo), ow = rem - oh * g.Wo;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    v[r] = make_uint4(0, 0, 0, 0);
    if (k0 + r < K) {
      const int ih0 = oh * g.stride - g.pad, iw0 = ow * g.stride - g.pad;
      const uint16_t* xb = x + (long)b * g.H * g.W * g.C;
      if (FORM != 2 && vec8) {
        const int ih = ih0 + dy0, iw = iw0 + dx0;
        if (ih >= 0 && ih < g.H && iw >= 0 && iw < g.W)
          v[r] = *(const uint4*)(xb + ((long)ih * g.W + iw) * g.C + ch0);
      } else {
        // every element load goes out unconditionally (padding taps read the image's first
        // element, then masked): loads behind a per-element branch were issued one after
        // another (the 3-channel first VGG16_bn layer: 456 -> 346 us)
        uint16_t t[8];
        int ch = ch0, dy = dy0, dx = dx0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = c0 + j;
          const int ih = ih0 + dy, iw = iw0 + dx;
          const bool in = col < ncols && ih >= 0 && ih < g.H && iw >= 0 && iw < g.W;
          const uint16_t e = xb[in ? ((long)ih * g.W + iw) * g.C + ch : 0];
          t[j] = in ? e : ((ones && col == ncols) ? (uint16_t)0x3f80 : (uint16_t)0);   // bf16 1.0
          if (col < ncols && ++ch == g.C) {
            ch = 0;
            if (++dx == g.kw) { dx = 0; ++dy; }
          }
        }
        v[r] = make_uint4(t[0] | ((uint32_t)t[1] << 16), t[2] | ((uint32_t)t[3] << 16),
                          t[4] | ((uint32_t)t[5] << 16), t[6] | ((uint32_t)t[7] << 16));
      }
    }
    if (++ow == g.Wo) {
      ow = 0;
      if (++oh == g.Ho) { oh = 0; ++b; }
    }
  }
}

// Patch staging: the patches gathered once into a zero-padded n x ldp buffer at the head of
// the caller's workspace (16-byte aligned rows, ldp = kh kw C rounded up to 8), which the EA
// and weight-gradient kernels then read as a plain row-major / K-major operand: 16-byte
// loads and the EA's pipelined stages instead of the per-row im2col address arithmetic.
// Done for every channel count that is not a multiple of 8 (the 3-channel first layer of
// an image network: one 2-byte load per element otherwise); for the EA also wherever the
// buffer takes at most kConvStageMax bytes (every VGG16_bn layer at batch 128, the largest
// at 144 MB: 64 MB measured 2.31 ms for the 13 layers' K-FAC work, 256 MB 2.25 ms; larger
// patch matrices stay implicit).  The weight gradient's 16-byte
// im2col gather is as fast as its ordinary K-major loader, so it stages only the former
// (staging every small layer measured 938 -> 1021 us for the VGG16_bn weight gradients,
// while the EA went 1755 -> 1495 us).
constexpr size_t kConvStageMax = 256u << 20;
__host__ __device__ inline int conv_patch_ld(const ConvGeom& g) { return (g.kh * g.kw * g.C + 7) / 8 * 8; }
inline size_t conv_patch_bytes(const ConvGeom& g, bool ea) {
  const size_t b = (size_t)g.B * g.Ho * g.Wo * conv_patch_ld(g) * sizeof(uint16_t);
  if (g.C % 8 == 0 && (!ea || b > kConvStageMax)) return 0;
  return (b + 255) / 256 * 256;
}

}  // namespace kfac
