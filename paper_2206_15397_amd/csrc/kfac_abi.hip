// C ABI of libkfac.so: argument validation, workspace layout and the launch sequences of
// the K-factor pipeline.  No device memory is allocated here; every buffer comes from the
// caller.
#include <cmath>
#include <cstring>
#include <utility>
#include "kernels.h"
#include "conv.h"

using namespace kfac;

#include "workspace.h"

using kfac::Bump;
using kfac::EigWs;
using kfac::round_up;

namespace {
inline kfac_status hip_status(hipError_t e) { return e == hipSuccess ? KFAC_OK : KFAC_EHIP; }
}  // namespace

extern "C" {

const char* kfac_status_string(kfac_status s) {
  switch (s) {
    case KFAC_OK: return "ok";
    case KFAC_EINVAL: return "invalid argument";
    case KFAC_EWORKSPACE: return "workspace too small";
    case KFAC_EHIP: return "HIP launch error";
    case KFAC_EUNSUPPORTED: return "unsupported configuration";
    case KFAC_ESCRATCH: return "problem needs more scratch than the allocation-free entry point's static buffer holds";
  }
  return "unknown status";
}

#ifndef KFAC_SRC_HASH
#define KFAC_SRC_HASH "unknown"
#endif
const char* kfac_build_info(void) {
  return "libkfac gfx950 (fp32/bf16 MFMA GEMM, fp64 CholeskyQR2 + tridiagonal eigensolver) src " KFAC_SRC_HASH;
}

kfac_status kfac_fill_identity(float* F, int64_t d, int64_t ldf, kfac_stream_t stream) {
  if (!F || d < 1 || ldf < d || d > (1 << 30)) return KFAC_EINVAL;
  return hip_status(launch_fill_identity(F, (int)d, ldf, (hipStream_t)stream));
}

size_t kfac_ea_update_workspace(int64_t d, int64_t n) {
  if (d < 1 || n < 0) return 0;
  return ea_workspace_bytes((int)d, n);
}

kfac_status kfac_ea_update(float* F, int64_t d, int64_t ldf, const void* X, kfac_dtype xtype, int64_t n,
                           int64_t d_in, int64_t ldx, int append_ones, float rho, float scale,
                           uint16_t* F_bf16, int64_t ldfb, void* workspace, size_t ws_bytes,
                           kfac_stream_t stream) {
  if (!F || d < 1 || ldf < d || n < 0 || d_in < 0) return KFAC_EINVAL;
  if (d != d_in + (append_ones ? 1 : 0)) return KFAC_EINVAL;
  if (n > 0 && (!X || ldx < d_in)) return KFAC_EINVAL;
  if (!(rho >= 0.f && rho < 1.f) || !(scale > 0.f) || !std::isfinite(scale)) return KFAC_EINVAL;
  if (xtype != KFAC_FP32 && xtype != KFAC_BF16) return KFAC_EINVAL;
  if (F_bf16 && ldfb < d) return KFAC_EINVAL;
  if (d > (1 << 20) || n > (1LL << 31) - 1) return KFAC_EUNSUPPORTED;
  if (ws_bytes == 0) workspace = nullptr;          // no workspace: no split-K
  if (workspace && ws_bytes < kfac_ea_update_workspace(d, n)) return KFAC_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (xtype == KFAC_FP32)
    return hip_status(launch_ea_f32(F, (int)d, ldf, (const float*)X, (int)n, (int)d_in, ldx, append_ones,
                                    rho, scale, F_bf16, ldfb, workspace, ws_bytes, s));
  return hip_status(launch_ea_bf16(F, (int)d, ldf, (const uint16_t*)X, (int)n, (int)d_in, ldx, append_ones,
                                   rho, scale, F_bf16, ldfb, workspace, ws_bytes, s));
}

kfac_status kfac_gaussian_omega(float* Omega, int64_t d, int64_t l, int64_t ldo, uint64_t seed,
                                uint64_t stream_id, uint32_t inversion_index, uint32_t* words,
                                kfac_stream_t stream) {
  if (d < 1 || l < 1 || (!Omega && !words) || (Omega && ldo < l)) return KFAC_EINVAL;
  if (d > (1 << 30) || l > (1 << 20)) return KFAC_EUNSUPPORTED;
  return hip_status(launch_omega((int)d, (int)l, (int)d, 0, seed, stream_id, inversion_index, nullptr, 0,
                                 nullptr, Omega, ldo, words, (hipStream_t)stream));
}

size_t kfac_rand_eig_workspace(int64_t d, int64_t r, int64_t p, int q, kfac_variant v, kfac_precision prec) {
  if (d < 1 || r < 1 || r > d || p < 0 || q < 0) return 0;
  (void)v;
  if (prec != KFAC_SKETCH_FP32 && prec != KFAC_SKETCH_BF16 && prec != KFAC_SKETCH_SPLIT) return 0;
  EigWs w(d, r, p, (int)prec, nullptr);
  return w.bytes;
}

kfac_status kfac_rand_eig(const float* F, int64_t d, int64_t ldf, const uint16_t* F_bf16, int64_t ldfb,
                          int64_t r, int64_t p, int q, uint64_t seed, uint64_t stream_id,
                          uint32_t inversion_index, kfac_variant v, kfac_precision prec, float* U,
                          int64_t ldu, float* D, void* workspace, size_t ws_bytes, int32_t* dev_status,
                          kfac_stream_t stream) {
  if (!F || !U || !D || !dev_status || !workspace) return KFAC_EINVAL;
  if (d < 1 || ldf < d || r < 1 || r > d || p < 0 || q < 0 || q > 16 || ldu < r) return KFAC_EINVAL;
  if (prec != KFAC_SKETCH_FP32 && prec != KFAC_SKETCH_BF16 && prec != KFAC_SKETCH_SPLIT) return KFAC_EINVAL;
  if (v != KFAC_SREVD && v != KFAC_RSVD) return KFAC_EINVAL;
  if (prec == KFAC_SKETCH_BF16 && (!F_bf16 || ldfb < d)) return KFAC_EINVAL;
  const bool rsvd = (v == KFAC_RSVD);
  const int64_t l = std::min<int64_t>(r + p, d);
  if (l > KFAC_MAX_SKETCH || d > (1 << 28)) return KFAC_EUNSUPPORTED;
  EigWs w(d, r, p, (int)prec, workspace);
  if (ws_bytes < w.bytes) return KFAC_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  int* st = (int*)dev_status;
  hipError_t e = hipSuccess;
#define CK(x) do { e = (x); if (e != hipSuccess) return KFAC_EHIP; } while (0)
  if (w.exact) {
    // l == d: the sketch spans R^d, Q = I; eigendecompose F itself, U = P[:, :r] (for the
    // RSVD variant this is also the SVD of B^T = F, F being symmetric PSD).
    CK(launch_small_eig(nullptr, 0, F, ldf, (int)d, (int)d, (int)r, w.A, w.V, w.diag, w.off, w.Z, w.scr, U,
                        ldu, D, w.Dd, st, s));
    CK(launch_sign_normalize(U, ldu, (int)d, (int)r, w.sval, w.sidx, s));
    return KFAC_OK;
  }
  const bool bf = (prec == KFAC_SKETCH_BF16);
  const bool sp = (prec == KFAC_SKETCH_SPLIT);
  const int L = (int)w.l_pad, n = (int)w.l, dd = (int)d;
  const long ldt = w.ldt;
  // Omega^T (l_pad x d), rows >= l zero
  CK(launch_omega(dd, n, dd, L, seed, stream_id, inversion_index, w.OmT, ldt, bf ? w.OmTb : nullptr, nullptr,
                  0, nullptr, s));
  // the whole-width kernels (all l_pad rows per workgroup) when l_pad fits them
  const bool whole = (bf || sp) && L <= kWholeWidthMaxM;
  auto f_times = [&](const float* At, const uint16_t* Atb, float* Out) -> hipError_t {
    // Out (L x d) = At (L x d) * F (d x d); F symmetric, so Out^T = F At^T.
    if (sp && whole)
      return launch_split(make_split_task(L, dd, dd, At, ldt, F, ldf, Out, ldt, w.skp, split_ksplit(dd, dd)), s);
    if (whole && dd >= 2048)
      return launch_skinny(make_skinny_task(L, dd, dd, Atb, ldt, F_bf16, ldfb, Out, ldt, w.skp,
                                            skinny_ksplit(dd, dd)), s);
    if (bf) return launch_gemm_bf16_nt(L, dd, dd, Atb, ldt, F_bf16, ldfb, Out, ldt, s);
    GemmP g{};
    g.M = L; g.N = dd; g.K = dd;
    g.A = At; g.lda = ldt; g.B = F; g.ldb = ldf;
    g.C = Out; g.ldc = ldt; g.alpha = 1.f; g.ones_col = -1;
    return launch_gemm(g, false, false, s);
  };
  // CholeskyQR2: Q1 = Y L1^{-T}, Q = Q1 L2^{-T} (fp64 Gram, Cholesky and triangular
  // product).  For l <= 288 the Cholesky also forms L^{-1} and the product is a plain
  // fp64 MFMA GEMM (out of place, so the basis ends in *cur); larger l uses blocked
  // forward substitution in place.  `cur` points at the buffer holding Q afterwards.
  // The orthonormalisations inside the power iteration take one pass (CholeskyQR): their
  // basis only has to span the same range with full rank, and the next product and the
  // final two-pass orthonormalisation restore orthonormality.
  float* cur = nullptr;
  auto cholqr = [&](float* Yt, float* other, uint16_t* Qtb, int npass) -> hipError_t {
    hipError_t x;
    float* src = Yt;
    float* dst = other;
    for (int pass = 0; pass < npass; ++pass) {
      uint16_t* qb = (pass == npass - 1) ? Qtb : nullptr;
      if ((x = launch_gram(src, ldt, src, ldt, L, dd, 1, w.part, w.G, L, st, s)) != hipSuccess) return x;
      if (L <= kCholInvMax) {
        int* keep = (pass == 1) ? w.fail + 1 : nullptr;     // second pass: kept out when not needed
        if ((x = launch_cholinv(w.G, L, n, dd, w.Wc, L, L, w.Li, st, w.fail, s, keep, kQrKeepTol)) != hipSuccess)
          return x;
        if ((x = launch_trmm(w.Wc, L, n, src, ldt, dd, dst, ldt, qb, ldt, L, s, keep)) != hipSuccess) return x;
        std::swap(src, dst);
      } else {
        if ((x = launch_cholesky(w.G, L, n, dd, w.Wc, L, w.Li, st, w.fail, s)) != hipSuccess) return x;
        if ((x = launch_trsm(w.Wc, L, w.Li, n, L, src, ldt, dd, src, ldt, qb, ldt, s)) != hipSuccess) return x;
      }
    }
    cur = src;
    return hipSuccess;
  };
  // sketch Y = F Omega, then orthonormalise
  CK(f_times(w.OmT, w.OmTb, w.Yt));
  // the bf16 copy of Q only where another bf16 product follows
  CK(cholqr(w.Yt, w.Qt, (bf && q > 0) ? w.Qtb : nullptr, q > 0 ? 1 : 2));
  for (int it = 0; it < q; ++it) {
    float* spare = (cur == w.Yt) ? w.Qt : w.Yt;
    CK(f_times(cur, w.Qtb, spare));
    CK(cholqr(spare, cur, (bf && it + 1 < q) ? w.Qtb : nullptr, it + 1 < q ? 1 : 2));
  }
  float* Qt = cur;
  float* Wt = (cur == w.Yt) ? w.Qt : w.Yt;
  // Rayleigh-Ritz: W = F Q (fp32 tiles; split-bf16 in the bf16-sketch mode), C = Q^T W (fp64)
  if (whole) {
    CK(launch_split(make_split_task(L, dd, dd, Qt, ldt, F, ldf, Wt, ldt, w.skp, split_ksplit(dd, dd)), s));
  } else {
    GemmP g{};
    g.M = L; g.N = dd; g.K = dd;
    g.A = Qt; g.lda = ldt; g.B = F; g.ldb = ldf;
    g.C = Wt; g.ldc = ldt; g.alpha = 1.f; g.ones_col = -1;
    CK(launch_gemm(g, false, false, s));
  }
  // SREVD (Alg. 3): C = Q^T W, eig(C) = P Lambda P^T, U = Q P[:, :r], D = Lambda[:r].
  // RSVD (Alg. 2, returning V as Sec. 2.2.2 prescribes for PSD factors): B^T = F Q = W; its
  // thin SVD W = V Sigma P^T from the eigendecomposition of the Gram W^T W = P Sigma^2 P^T
  // (fp64), V = W P Sigma^{-1}; U = V[:, :r], D = Sigma[:r].
  if (rsvd) CK(launch_gram(Wt, ldt, Wt, ldt, L, dd, 1, w.part, w.G, L, st, s));
  else CK(launch_gram(Qt, ldt, Wt, ldt, L, dd, 0, w.part, w.G, L, st, s));
  CK(launch_small_eig(w.G, L, nullptr, 0, n, L, (int)r, w.A, w.V, w.diag, w.off, w.Z, w.scr, w.P, r, D, w.Dd,
                      st, s, rsvd ? 1 : 0));
  // U = Q P[:, :r] (SREVD) or W P[:, :r] Sigma^{-1} (RSVD; P already scaled); the left
  // operand is stored transposed (l_pad x d, i.e. K x M)
  {
    GemmP g{};
    g.M = dd; g.N = (int)r; g.K = n;
    g.A = rsvd ? Wt : Qt; g.lda = ldt; g.B = w.P; g.ldb = r;
    g.C = U; g.ldc = ldu; g.alpha = 1.f; g.ones_col = -1;
    CK(launch_gemm(g, true, false, s));
  }
  CK(launch_sign_normalize(U, ldu, dd, (int)r, w.sval, w.sidx, s));
#undef CK
  return KFAC_OK;
}

size_t kfac_precondition_workspace(int64_t d_g, int64_t d_a, int64_t r_a, int64_t r_g) {
  if (d_g < 1 || d_a < 1 || r_a < 1 || r_g < 1) return 0;
  Bump b(nullptr);
  b.take<float>(d_g * r_a);
  b.take<float>(d_g * d_a);
  b.take<float>(r_g * d_a);
  return b.off + kAlign;
}

kfac_status kfac_precondition(const float* J, int64_t d_g, int64_t d_a, int64_t ldj, const float* U_a,
                              int64_t ldua, const float* D_a, int64_t r_a, const float* U_g, int64_t ldug,
                              const float* D_g, int64_t r_g, float lambda, float* S, int64_t lds,
                              void* workspace, size_t ws_bytes, kfac_stream_t stream) {
  if (!J || !U_a || !D_a || !U_g || !D_g || !S || !workspace) return KFAC_EINVAL;
  if (d_g < 1 || d_a < 1 || ldj < d_a || lds < d_a) return KFAC_EINVAL;
  if (r_a < 1 || r_a > d_a || r_g < 1 || r_g > d_g || ldua < r_a || ldug < r_g) return KFAC_EINVAL;
  if (!(lambda > 0.f) || !std::isfinite(lambda)) return KFAC_EINVAL;
  if ((const void*)S == (const void*)J) return KFAC_EINVAL;
  if (d_g > (1 << 28) || d_a > (1 << 28)) return KFAC_EUNSUPPORTED;
  if (ws_bytes < kfac_precondition_workspace(d_g, d_a, r_a, r_g)) return KFAC_EWORKSPACE;
  Bump b(workspace);
  float* T1 = b.take<float>(d_g * r_a);
  float* M = b.take<float>(d_g * d_a);
  float* T2 = b.take<float>(r_g * d_a);
  hipStream_t s = (hipStream_t)stream;
  const float inv_lam = 1.0f / lambda;
  hipError_t e;
  {  // T1 = J U_a diag(f_a)
    GemmP g{};
    g.M = (int)d_g; g.N = (int)r_a; g.K = (int)d_a;
    g.A = J; g.lda = ldj; g.B = U_a; g.ldb = ldua; g.C = T1; g.ldc = r_a;
    g.alpha = 1.f; g.colD = D_a; g.lam = lambda; g.ones_col = -1;
    if ((e = launch_gemm(g, false, false, s)) != hipSuccess) return KFAC_EHIP;
  }
  {  // M = T1 U_a^T + J / lambda
    GemmP g{};
    g.M = (int)d_g; g.N = (int)d_a; g.K = (int)r_a;
    g.A = T1; g.lda = r_a; g.B = U_a; g.ldb = ldua; g.C = M; g.ldc = d_a;
    g.alpha = 1.f; g.X = J; g.ldx = ldj; g.beta = inv_lam; g.ones_col = -1;
    if ((e = launch_gemm(g, false, true, s)) != hipSuccess) return KFAC_EHIP;
  }
  {  // T2 = diag(f_g) U_g^T M
    GemmP g{};
    g.M = (int)r_g; g.N = (int)d_a; g.K = (int)d_g;
    g.A = U_g; g.lda = ldug; g.B = M; g.ldb = d_a; g.C = T2; g.ldc = d_a;
    g.alpha = 1.f; g.rowD = D_g; g.lam = lambda; g.ones_col = -1;
    if ((e = launch_gemm(g, true, false, s)) != hipSuccess) return KFAC_EHIP;
  }
  {  // S = U_g T2 + M / lambda
    GemmP g{};
    g.M = (int)d_g; g.N = (int)d_a; g.K = (int)r_g;
    g.A = U_g; g.lda = ldug; g.B = T2; g.ldb = d_a; g.C = S; g.ldc = lds;
    g.alpha = 1.f; g.X = M; g.ldx = d_a; g.beta = inv_lam; g.ones_col = -1;
    if ((e = launch_gemm(g, false, false, s)) != hipSuccess) return KFAC_EHIP;
  }
  return KFAC_OK;
}

kfac_status kfac_linear_forward(const uint16_t* x, int64_t n, int64_t d_in, int64_t ldx, const uint16_t* W,
                                int64_t d_out, int64_t ldw, const float* bias, uint16_t* y, int64_t ldy,
                                kfac_stream_t stream) {
  if (!W || (n > 0 && (!x || !y))) return KFAC_EINVAL;
  if (n < 0 || d_in < 1 || d_out < 1 || ldx < d_in || ldw < d_in || ldy < d_out) return KFAC_EINVAL;
  if (n == 0) return KFAC_OK;
  if (n > INT32_MAX || d_in > INT32_MAX || d_out > INT32_MAX) return KFAC_EUNSUPPORTED;
  return hip_status(launch_linear_forward(x, (int)n, (int)d_in, ldx, W, (int)d_out, ldw, bias, y, ldy,
                                          (hipStream_t)stream));
}

kfac_status kfac_linear_backward(const uint16_t* g, int64_t n, int64_t d_out, int64_t ldg, const uint16_t* x,
                                 int64_t d_in, int64_t ldx, const uint16_t* W, int64_t ldw, uint16_t* dx,
                                 int64_t lddx, float* dWb, int64_t lddw, int with_bias, float* Gamma, int64_t ldgam,
                                 uint16_t* Gamma_bf16, int64_t ldgb, float rho, float scale, kfac_stream_t stream) {
  if (!W || !dWb || (n > 0 && (!g || !x))) return KFAC_EINVAL;
  if (n < 0 || d_in < 1 || d_out < 1 || ldg < d_out || ldx < d_in || ldw < d_in) return KFAC_EINVAL;
  if (lddw < d_in + (with_bias ? 1 : 0)) return KFAC_EINVAL;
  if (dx && lddx < d_in) return KFAC_EINVAL;
  if (Gamma) {
    if (ldgam < d_out || !(rho >= 0.f && rho < 1.f) || !(scale > 0.f)) return KFAC_EINVAL;
    if (Gamma_bf16 && ldgb < d_out) return KFAC_EINVAL;
  }
  if (n > INT32_MAX || d_in > INT32_MAX || d_out > INT32_MAX) return KFAC_EUNSUPPORTED;
  return hip_status(launch_linear_backward(g, (int)n, (int)d_out, ldg, x, (int)d_in, ldx, W, ldw, dx, lddx, dWb, lddw,
                                           with_bias ? 1 : 0, Gamma, ldgam, Gamma_bf16, ldgb, rho, scale,
                                           (hipStream_t)stream));
}

}  // extern "C"

namespace {
// Validated device geometry of a kfac_conv_geom (false: invalid or beyond 32-bit indexing).
bool conv_geom(const kfac_conv_geom* g, const void* x, ConvGeom& cv, kfac_status& err) {
  err = KFAC_EINVAL;
  if (!g || g->batch < 1 || g->height < 1 || g->width < 1 || g->channels < 1 || g->kh < 1 || g->kw < 1 ||
      g->pad < 0 || g->stride < 1)
    return false;
  const int64_t ho = (g->height + 2 * g->pad - g->kh) / g->stride + 1;
  const int64_t wo = (g->width + 2 * g->pad - g->kw) / g->stride + 1;
  if (g->height + 2 * g->pad < g->kh || g->width + 2 * g->pad < g->kw || ho < 1 || wo < 1) return false;
  const int64_t lim = (1LL << 31) - 1;
  if (g->batch * g->height * g->width * g->channels > lim || g->batch * ho * wo > lim ||
      g->kh * g->kw * g->channels > lim) {
    err = KFAC_EUNSUPPORTED;
    return false;
  }
  cv = ConvGeom{(int)g->batch, (int)g->height, (int)g->width, (int)g->channels, (int)g->kh, (int)g->kw,
                (int)g->pad, (int)g->stride, (int)ho, (int)wo,
                (g->channels % 8 == 0 && (((uintptr_t)x) & 15) == 0) ? 1 : 0,
                conv_divisor((int)g->channels), conv_divisor((int)g->kw), conv_divisor((int)(ho * wo)),
                conv_divisor((int)wo)};
  return true;
}
}  // namespace

extern "C" {

size_t kfac_conv_ea_update_workspace(int64_t d, const kfac_conv_geom* geom) {
  ConvGeom cv;
  kfac_status err;
  if (d < 1 || !conv_geom(geom, nullptr, cv, err)) return 0;
  return ea_workspace_bytes((int)d, (long)cv.B * cv.Ho * cv.Wo) + conv_patch_bytes(cv, true);
}

kfac_status kfac_conv_ea_update(float* F, int64_t d, int64_t ldf, const uint16_t* x, const kfac_conv_geom* geom,
                                int append_ones, float rho, float scale, uint16_t* F_bf16, int64_t ldfb,
                                void* workspace, size_t ws_bytes, kfac_stream_t stream) {
  ConvGeom cv;
  kfac_status err;
  if (!F || !x || d < 1 || ldf < d) return KFAC_EINVAL;
  if (!conv_geom(geom, x, cv, err)) return err;
  if (d != (int64_t)cv.kh * cv.kw * cv.C + (append_ones ? 1 : 0)) return KFAC_EINVAL;
  if (!(rho >= 0.f && rho < 1.f) || !(scale > 0.f) || !std::isfinite(scale)) return KFAC_EINVAL;
  if (F_bf16 && ldfb < d) return KFAC_EINVAL;
  if (d > (1 << 20)) return KFAC_EUNSUPPORTED;
  if (ws_bytes == 0) workspace = nullptr;
  if (workspace && ws_bytes < kfac_conv_ea_update_workspace(d, geom)) return KFAC_EWORKSPACE;
  return hip_status(launch_ea_bf16_conv(F, (int)d, ldf, x, cv, append_ones ? 1 : 0, rho, scale, F_bf16, ldfb,
                                        workspace, ws_bytes, (hipStream_t)stream));
}

size_t kfac_conv_backward_weight_workspace(int64_t c_out, const kfac_conv_geom* geom, int with_bias) {
  ConvGeom cv;
  kfac_status err;
  if (c_out < 1 || c_out > (1 << 20) || !conv_geom(geom, nullptr, cv, err)) return 0;
  return conv_backward_weight_ws_bytes((int)c_out, (long)cv.B * cv.Ho * cv.Wo,
                                       cv.kh * cv.kw * cv.C + (with_bias ? 1 : 0)) + conv_patch_bytes(cv, false);
}

kfac_status kfac_conv_backward_weight(const uint16_t* g, int64_t c_out, const uint16_t* x,
                                      const kfac_conv_geom* geom, float* dWb, int64_t lddw, int with_bias,
                                      float* Gamma, int64_t ldgam, uint16_t* Gamma_bf16, int64_t ldgb, float rho,
                                      float scale, void* workspace, size_t ws_bytes, kfac_stream_t stream) {
  ConvGeom cv;
  kfac_status err;
  if (!g || !x || !dWb || c_out < 1) return KFAC_EINVAL;
  if (!conv_geom(geom, x, cv, err)) return err;
  if (lddw < (int64_t)cv.kh * cv.kw * cv.C + (with_bias ? 1 : 0)) return KFAC_EINVAL;
  if (Gamma) {
    if (ldgam < c_out || !(rho >= 0.f && rho < 1.f) || !(scale > 0.f)) return KFAC_EINVAL;
    if (Gamma_bf16 && ldgb < c_out) return KFAC_EINVAL;
  }
  if (c_out > (1 << 20)) return KFAC_EUNSUPPORTED;
  if (ws_bytes == 0) workspace = nullptr;
  if (workspace && ws_bytes < kfac_conv_backward_weight_workspace(c_out, geom, with_bias)) return KFAC_EWORKSPACE;
  return hip_status(launch_conv_backward_weight(g, x, cv, (int)c_out, dWb, lddw, with_bias ? 1 : 0, Gamma, ldgam,
                                                Gamma_bf16, ldgb, rho, scale, workspace, ws_bytes,
                                                (hipStream_t)stream));
}

}  // extern "C"
