// Device-side helpers shared by the gfx950 kernels of libkfac: MFMA fragment types,
// bf16 rounding, wavefront reductions and the Philox4x32-10 generator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>
#include <type_traits>

namespace kfac {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// fp32 -> bf16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// All-ones or zero mask the compiler cannot see through: `load & mask` keeps the load
// unconditional (from a clamped, valid address) instead of sinking it into a branch.
__device__ __forceinline__ uint32_t opaque_mask(bool keep) {
  uint32_t m = keep ? 0xffffffffu : 0u;
  asm("" : "+v"(m));       // not volatile: no side effects, so memory is not re-read around it
  return m;
}
// 16-byte load through a global-address-space pointer (a global_load, which unlike a
// flat load does not hold back the LDS wait counter); p must be 16-byte aligned.
__device__ __forceinline__ uint4 gload16(const void* p) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gp;
  const u32x4 v = *(gp)__builtin_assume_aligned(p, 16);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t gload4(const void* p) {
  typedef const uint32_t __attribute__((address_space(1)))* gp;
  return *(gp)p;
}
__device__ __forceinline__ uint4 and_mask(uint4 v, uint32_t m) { return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// LDS writes of this wavefront visible to its own later LDS reads (no workgroup barrier):
// wait for the wavefront's outstanding LDS operations only, so global stores keep flowing,
// and keep the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_order() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Two fp32 -> packed bf16 (a in the low half), round to nearest even: one
// v_cvt_pk_bf16_f32 on gfx950.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const f32x2 x = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2));
}

// Cross-lane moves on the DPP network (no LDS round trip).  Control codes of the GFX9
// DPP encoding: quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, row_mirror = 0x140,
// row_half_mirror = 0x141, row_bcast:15 = 0x142, row_bcast:31 = 0x143.  Lanes of rows
// outside ROW_MASK keep `old`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double old, double src) {
  const long long o = __builtin_bit_cast(long long, old), v = __builtin_bit_cast(long long, src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROW_MASK, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, src), CTRL, ROW_MASK, 0xf,
                                                               false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_t(double old, double src) { return dpp_f64<CTRL, ROW_MASK>(old, src); }
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_t(float old, float src) { return dpp_f32<CTRL, ROW_MASK>(old, src); }

// DPP moves whose lanes outside ROW_MASK are left undefined (no `old` value to set up
// first): for reductions whose result is only read in the written lanes.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_any(double src) {
  const long long v = __builtin_bit_cast(long long, src);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), CTRL, ROW_MASK, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_any(float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, src), CTRL, ROW_MASK, 0xf, false));
}

// Sum over each row of 16 lanes; every lane of the row receives it.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v += dpp_any<0xB1>(v);
  v += dpp_any<0x4E>(v);
  v += dpp_any<0x141>(v);
  v += dpp_any<0x140>(v);
  return v;
}

// Sum over each half wavefront (lanes 0-31, 32-63); the result is valid in lanes 16-31
// and 48-63 (rows 1 and 3) only.
template <typename T>
__device__ __forceinline__ T half_sum_hi(T v) {
  v = row16_sum(v);
  v += dpp_any<0x142, 0xA>(v);
  return v;
}

__device__ __forceinline__ double readlane_t(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_t(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the wavefront (all 64 lanes active), returned to every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v = half_sum_hi(v);
  v += dpp_any<0x143, 0xC>(v);          // row 3 now holds the total
  return readlane_t(v, 63);
}

// 1 / sqrt(x) for normal x > 0: the hardware estimate refined by two Newton steps
// y <- y (3/2 - x y^2 / 2) (quadratic convergence from ~2^-22 to full fp64 precision).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32 Philox
// bijection; multipliers M0, M1 and Weyl key increments W0, W1.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// Uniform in (0,1) with 24 significant bits (exact in fp32 and fp64).
__device__ __forceinline__ double philox_uniform(uint32_t w) {
  return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

// Four N(0,1) values for counter (row, group, stream, inversion): two Box-Muller pairs,
// evaluated in fp64.
__device__ __forceinline__ void gaussian4(uint32_t row, uint32_t group, uint32_t stream,
                                          uint32_t inv, uint32_t k0, uint32_t k1, double z[4],
                                          uint32_t words[4]) {
  uint32_t c[4] = {row, group, stream, inv};
  philox4x32_10(c, k0, k1);
#pragma unroll
  for (int t = 0; t < 4; ++t) words[t] = c[t];
  double u0 = philox_uniform(c[0]), u1 = philox_uniform(c[1]);
  double u2 = philox_uniform(c[2]), u3 = philox_uniform(c[3]);
  double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  double s1, c1, s3, c3;
  sincospi(2.0 * u1, &s1, &c1);
  sincospi(2.0 * u3, &s3, &c3);
  z[0] = r01 * c1; z[1] = r01 * s1; z[2] = r23 * c3; z[3] = r23 * s3;
}

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1.  Register arrays
// indexed with the constant stay in registers (no dynamic indexing, no scratch).
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace kfac
