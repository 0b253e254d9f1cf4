/*
 * kfac.h -- C ABI of libkfac.so, the MI355X (gfx950) K-factor pipeline of Randomized
 * K-FAC (Puiu, "Randomized K-FACs: Speeding up K-FAC with Randomized Numerical Linear
 * Algebra", arXiv 2206.15397).
 *
 * Conventions shared by every entry point
 *  - Every data pointer is a DEVICE pointer into memory the caller allocated and owns
 *    (hipMalloc / a PyTorch tensor).  The library never allocates device memory and
 *    never frees caller memory; scratch comes from the caller through `workspace`
 *    (size from the matching *_workspace query; a larger buffer is fine).
 *  - Matrices are row-major; a leading dimension (ld*) is the distance in elements
 *    between consecutive rows and must be >= the row length.
 *  - All calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL is the
 *    default stream).  A call returns after enqueueing; results are ready once the
 *    stream has been synchronised.
 *  - Argument errors are reported synchronously as KFAC_EINVAL before anything is
 *    enqueued; KFAC_EWORKSPACE if the workspace is smaller than the query says;
 *    KFAC_EHIP if a launch failed; KFAC_EUNSUPPORTED for sizes beyond the compiled
 *    limits (sketch width l = min(r+p, d) > KFAC_MAX_SKETCH).
 *  - Conditions only the device can see (Cholesky breakdown, non-finite values,
 *    eigensolver non-convergence) are OR-ed as bits into *dev_status (int32, device
 *    memory, caller clears it); read it after synchronising the stream.
 *  - Calls on different streams with disjoint buffers may run concurrently.  Calls that
 *    share a workspace must be ordered on one stream.
 */
#ifndef KFAC_H
#define KFAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KFAC_OK = 0,
  KFAC_EINVAL = 1,
  KFAC_EWORKSPACE = 2,
  KFAC_EHIP = 3,
  KFAC_EUNSUPPORTED = 4,
  KFAC_ESCRATCH = 5     /* the allocation-free entry point's static scratch is too small */
} kfac_status;

typedef enum { KFAC_FP32 = 0, KFAC_BF16 = 1 } kfac_dtype;

/* Which randomized decomposition of the symmetric PSD factor F, after the same range
 * finder (Omega, sketch, power iterations, orthonormal Q):
 *  KFAC_SREVD  Alg. 3 (used by SRE-KFAC, Alg. 5): C = Q^T F Q, C = P Lambda P^T,
 *              U = Q P[:, :r], D = Lambda[:r].
 *  KFAC_RSVD   Alg. 2 (used by RS-KFAC, Alg. 4) returning the V factor, which Sec. 2.2.2
 *              prescribes for PSD factors: B = Q^T F, B^T = F Q = V_B Sigma U_B^T (thin
 *              SVD), U = V_B[:, :r], D = Sigma[:r].  The SVD is taken through the fp64
 *              eigendecomposition of the l x l Gram (FQ)^T (FQ) = U_B Sigma^2 U_B^T,
 *              V_B = F Q U_B Sigma^{-1}; columns with Sigma_k = 0 come out zero. */
typedef enum { KFAC_SREVD = 0, KFAC_RSVD = 1 } kfac_variant;

/* Precision of the sketch and power-iteration products F*Omega, F*Q (Alg. 3 "Compute
 * X Omega" and the power iterations of Sec. 2.2).
 *  KFAC_SKETCH_FP32   fp32 operands on fp32 MFMA.
 *  KFAC_SKETCH_BF16   bf16 operands (a bf16 copy of F supplied by the caller, e.g. the
 *                     shadow written by kfac_ea_update, and bf16 Omega / Q) with fp32
 *                     accumulation.  Rounding F to bf16 perturbs it by about 2^-9 ||F||,
 *                     which moves the Ritz values near the rank cut by up to that much
 *                     relative to lambda_r: accurate to the 5e-3 gate only where
 *                     lambda_r >> 2^-9 ||F|| (e.g. EA factors with the identity floor).
 *  KFAC_SKETCH_SPLIT  fp32 F and fp32 Omega / Q, each entering bf16 MFMAs as a pair
 *                     hi = bf16(v), lo = bf16(v - hi); three bf16 MFMAs per product
 *                     (hi*hi + hi*lo + lo*hi) with fp32 accumulation: fp32-class accuracy
 *                     at bf16-MFMA speed, no bf16 copy of F needed.
 * In every mode the Gram matrices, Cholesky factors and the (r+p)x(r+p) eigensolve are
 * fp64; the Rayleigh-Ritz product F*Q is fp32 MFMA (FP32 mode) or split-bf16 (the two
 * bf16 modes). */
typedef enum { KFAC_SKETCH_FP32 = 0, KFAC_SKETCH_BF16 = 1, KFAC_SKETCH_SPLIT = 2 } kfac_precision;

#define KFAC_MAX_SKETCH 512   /* largest l = min(r+p, d) handled by the fp64 eigensolver */

/* device status bits (OR-ed into *dev_status) */
#define KFAC_DS_CHOL_SHIFTED 0x1  /* a CholeskyQR Gram was not numerically SPD; a shift was
                                      added (shifted CholeskyQR) and the pass repeated      */
#define KFAC_DS_CHOL_FAILED  0x2  /* breakdown even after the shift: outputs are undefined  */
#define KFAC_DS_NONFINITE    0x4  /* NaN/Inf met in a Gram or projected matrix               */
#define KFAC_DS_EIG_NOCONV   0x8  /* small eigensolver hit its iteration cap                 */

typedef void* kfac_stream_t; /* hipStream_t */

/* Text for a status code (static storage, never NULL). */
const char* kfac_status_string(kfac_status s);

/* Library / device build information: target, kernel families and "src <hash>", a hash of
 * the sources and build flags the library was compiled from.  Static string. */
const char* kfac_build_info(void);

/*
 * kfac_fill_identity -- F <- I (d x d, fp32, ldf).  The EA K-factors start from the
 * identity (Alg. 1: the EA factors at step -1 are I).
 */
kfac_status kfac_fill_identity(float* F, int64_t d, int64_t ldf, kfac_stream_t stream);

/*
 * kfac_ea_update -- exponential-average K-factor update (Alg. 1, forward line
 * A_k <- rho A_{k-1} + (1-rho) A A^T and backward line for Gamma; matrix form in Sec. 3):
 *
 *     F <- rho * F + (1 - rho) * scale * Xh^T Xh,     Xh = [X | 1] if append_ones else X
 *
 *  F        d x d fp32 (ldf >= d), symmetric on entry; both triangles are written, so
 *           it stays exactly symmetric.  d must equal d_in + append_ones.
 *  X        n x d_in activations (forward factor: layer inputs a; backward factor:
 *           back-propagated pre-activation gradients g), one sample per row, ldx >= d_in,
 *           dtype xtype (fp32 or bf16).  n == 0 means "no samples": F <- rho F.
 *  rho      EA decay in [0, 1).   scale > 0, normally 1/n.
 *  F_bf16   optional (NULL allowed) bf16 shadow of the updated F, d x d, ldfb >= d,
 *           rounded to nearest even; it feeds the bf16 sketch of kfac_rand_eig.
 *  workspace/ws_bytes: scratch for split-K partial sums; size from
 *           kfac_ea_update_workspace(d, n).  A NULL/0 workspace is allowed and disables
 *           split-K (slower for small d and large n, identical results up to the
 *           summation order).
 */
size_t kfac_ea_update_workspace(int64_t d, int64_t n);
kfac_status kfac_ea_update(float* F, int64_t d, int64_t ldf,
                           const void* X, kfac_dtype xtype, int64_t n, int64_t d_in, int64_t ldx,
                           int append_ones, float rho, float scale,
                           uint16_t* F_bf16, int64_t ldfb,
                           void* workspace, size_t ws_bytes, kfac_stream_t stream);

/*
 * kfac_gaussian_omega -- the Gaussian test matrix Omega of Alg. 2/3 ("Sample Gaussian
 * Matrix"), materialised for inspection.  Omega_ij for row i < d, column j < l comes
 * from Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 * (i, j/4, stream_id mod 2^32, inversion_index); the four words w_t give uniforms
 * u_t = ((w_t >> 9) + 1/2) 2^-23 and the Box-Muller pairs
 * (z0,z1) = sqrt(-2 ln u0)(cos 2pi u1, sin 2pi u1), (z2,z3) likewise from (u2,u3);
 * Omega_ij = z_{j mod 4}.  kfac_rand_eig draws the same Omega internally.
 *  Omega    d x l fp32, ldo >= l (may be NULL if only words are wanted).
 *  words    optional (NULL allowed) d x ceil(l/4) x 4 uint32 raw Philox words.
 */
kfac_status kfac_gaussian_omega(float* Omega, int64_t d, int64_t l, int64_t ldo,
                                uint64_t seed, uint64_t stream_id, uint32_t inversion_index,
                                uint32_t* words, kfac_stream_t stream);

/*
 * kfac_rand_eig -- randomized low-rank eigendecomposition of one K-factor (SREVD, Alg. 3,
 * or RSVD, Alg. 2, see kfac_variant; with the power iterations of Sec. 2.2), replacing the
 * cubic full eig of Alg. 1:
 *   l = min(r + p, d).  If l < d: Y = F Omega (d x l); Q = orth(Y) by CholeskyQR2
 *   (fp64 Gram and Cholesky); q times: Y = F Q, Q = orth(Y).  If l == d: Q = I.
 *   SREVD: C = Q^T F Q (fp64, symmetrised); C = P diag(Lambda) P^T (fp64, descending);
 *   U = Q P[:, :r], D = Lambda[:r].  RSVD: W = F Q, W^T W = P diag(Sigma^2) P^T (fp64),
 *   U = W P[:, :r] Sigma^{-1}, D = Sigma[:r] (at l == d both are the eig of F).  Each
 *   column of U is signed so that its largest-magnitude entry is positive (ties: lowest
 *   row).
 *  F        d x d fp32 symmetric PSD factor (ldf >= d).
 *  F_bf16   bf16 copy of F (ldfb >= d); required iff prec == KFAC_SKETCH_BF16.
 *  r        target rank, 1 <= r <= d.  p >= 0 oversampling.  0 <= q <= 16 power its.
 *  seed, stream_id, inversion_index: select Omega (see kfac_gaussian_omega).
 *  U        d x r fp32 output (ldu >= r), orthonormal columns.   D: r fp32, descending.
 *  workspace: kfac_rand_eig_workspace(d, r, p, q, v, prec) bytes.
 *  dev_status: device int32 that receives KFAC_DS_* bits (required).
 */
size_t kfac_rand_eig_workspace(int64_t d, int64_t r, int64_t p, int q,
                               kfac_variant v, kfac_precision prec);
kfac_status kfac_rand_eig(const float* F, int64_t d, int64_t ldf,
                          const uint16_t* F_bf16, int64_t ldfb,
                          int64_t r, int64_t p, int q,
                          uint64_t seed, uint64_t stream_id, uint32_t inversion_index,
                          kfac_variant v, kfac_precision prec,
                          float* U, int64_t ldu, float* D,
                          void* workspace, size_t ws_bytes, int32_t* dev_status,
                          kfac_stream_t stream);

/*
 * kfac_rand_eig_noalloc -- kfac_rand_eig with no workspace argument and no allocation,
 * for callers that cannot allocate device memory: code under hipGraph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same operation, arguments, outputs and
 * errors as kfac_rand_eig; the scratch is a static device array of
 * KFAC_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until the process
 * ends (its address is looked up once per device, on the first call with that device
 * current).  Returns KFAC_ESCRATCH, before enqueueing anything, when
 * kfac_rand_eig_workspace(d, r, p, q, v, prec) exceeds that size (e.g. d above ~8192 with
 * the bf16 sketch at l = 272).  All calls on one GPU share the array: calls that overlap
 * in time (different streams, host threads) race; calls on one stream are ordered.
 */
#define KFAC_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
kfac_status kfac_rand_eig_noalloc(const float* F, int64_t d, int64_t ldf,
                                  const uint16_t* F_bf16, int64_t ldfb,
                                  int64_t r, int64_t p, int q,
                                  uint64_t seed, uint64_t stream_id, uint32_t inversion_index,
                                  kfac_variant v, kfac_precision prec,
                                  float* U, int64_t ldu, float* D,
                                  int32_t* dev_status, kfac_stream_t stream);

/*
 * kfac_precondition -- damped low-rank inverse application (Sec. 4.1 identity, the M and
 * S lines of Alg. 4; Alg. 5 uses V = U):
 *   f_a = 1/(D_a + lambda) - 1/lambda,  f_g likewise;
 *   M = J U_a diag(f_a) U_a^T + J / lambda;
 *   S = U_g diag(f_g) U_g^T M + M / lambda   ( = (G+lambda I)^{-1} J (A+lambda I)^{-1}
 *       when U, D are exact eigenpairs of full rank).
 *  J        d_g x d_a fp32 gradient Mat(g) (ldj >= d_a): rows = backward (Gamma) side,
 *           columns = forward (A) side.
 *  U_a, D_a d_a x r_a (ldua >= r_a) and r_a;   U_g, D_g  d_g x r_g (ldug >= r_g), r_g.
 *  lambda   > 0.   S: d_g x d_a fp32 output (lds >= d_a); must not alias J.
 *  workspace: kfac_precondition_workspace(d_g, d_a, r_a, r_g) bytes.
 */
size_t kfac_precondition_workspace(int64_t d_g, int64_t d_a, int64_t r_a, int64_t r_g);
kfac_status kfac_precondition(const float* J, int64_t d_g, int64_t d_a, int64_t ldj,
                              const float* U_a, int64_t ldua, const float* D_a, int64_t r_a,
                              const float* U_g, int64_t ldug, const float* D_g, int64_t r_g,
                              float lambda, float* S, int64_t lds,
                              void* workspace, size_t ws_bytes, kfac_stream_t stream);


/*
 * K-FAC linear layer (Alg. 1: the forward pass that provides the activations a of the
 * forward factor, and the backward pass that provides the weight gradient and the
 * back-propagated gradients g of the backward factor).  bf16 operands on MFMA with fp32
 * accumulation; row-major; a batch row per sample.
 *
 * kfac_linear_forward:   y = x W^T + b.
 *  x  n x d_in bf16 (ldx >= d_in);  W  d_out x d_in bf16 (ldw >= d_in);
 *  bias  d_out fp32 or NULL;  y  n x d_out bf16 output (ldy >= d_out).
 *
 * kfac_linear_backward:  one call for the layer's backward:
 *   dx = g W                                     (bf16, skipped when dx == NULL)
 *   [dW | db] = g^T [x | 1]                      (fp32 d_out x (d_in + with_bias), lddw >=
 *                                                 d_in + with_bias; column d_in holds db)
 *   Gamma <- rho Gamma + (1 - rho) scale g^T g   (Alg. 1's EA of the backward factor, fused
 *                                                 into the dW launch; skipped when Gamma ==
 *                                                 NULL; both triangles + optional bf16 shadow)
 *  g  n x d_out bf16 (ldg >= d_out); x as in the forward; W as in the forward.
 *  Gamma  d_out x d_out fp32 (ldgam >= d_out), Gamma_bf16 nullable (ldgb >= d_out).
 *  rho in [0, 1), scale > 0 (typically 1/n).  n == 0 gives dW = 0 and Gamma <- rho Gamma
 *  (g, x, dx may then be NULL); the forward with n == 0 does nothing.
 * Errors: KFAC_EINVAL for null required pointers, non-positive sizes or short leading
 * dimensions; KFAC_EHIP when a launch fails.
 */
kfac_status kfac_linear_forward(const uint16_t* x, int64_t n, int64_t d_in, int64_t ldx,
                                const uint16_t* W, int64_t d_out, int64_t ldw, const float* bias,
                                uint16_t* y, int64_t ldy, kfac_stream_t stream);
kfac_status kfac_linear_backward(const uint16_t* g, int64_t n, int64_t d_out, int64_t ldg,
                                 const uint16_t* x, int64_t d_in, int64_t ldx,
                                 const uint16_t* W, int64_t ldw,
                                 uint16_t* dx, int64_t lddx,
                                 float* dWb, int64_t lddw, int with_bias,
                                 float* Gamma, int64_t ldgam, uint16_t* Gamma_bf16, int64_t ldgb,
                                 float rho, float scale, kfac_stream_t stream);

/*
 * K-FAC convolution layer (the KFC factors that K-FAC uses for convolutions, Sec. 2.1; the
 * paper's VGG16_bn experiments of Sec. 5 are convolutional).  The input factor of a
 * convolution is the EA of the im2col patches of its input: one row per output position
 * (b, oh, ow), the columns ordered (dy, dx, c) -- tap-major, channel-minor -- plus the bias
 * column.  The patches are read straight from the NHWC input by the kernels' loaders and are
 * never materialised.
 *  kfac_conv_geom: input x is batch x height x width x channels, NHWC bf16 (contiguous);
 *  kernel kh x kw, zero padding `pad`, stride `stride`; output height
 *  (height + 2 pad - kh) / stride + 1, width likewise.  n = batch * out_h * out_w rows.
 *
 * kfac_conv_ea_update: F <- rho F + (1 - rho) scale [P | 1]^T [P | 1] (as kfac_ea_update
 *   with X = P, the n x (kh kw channels) patch matrix); d = kh kw channels + append_ones.
 *   workspace: kfac_conv_ea_update_workspace(d, geom) bytes (NULL / 0 disables split-K).
 * kfac_conv_backward_weight: [dW | db] = g^T [P | 1] (fp32, c_out x (kh kw channels +
 *   with_bias), lddw >= that; dW's columns in the patch order above, db last) from the output
 *   gradient g (n x c_out, i.e. NHWC batch x out_h x out_w x c_out, bf16), with the
 *   backward factor's EA Gamma <- rho Gamma + (1 - rho) scale g^T g fused into the same launch
 *   (skipped when Gamma == NULL; Gamma_bf16 nullable).  The contraction over the n positions
 *   is split into K slices whose raw sums go to the workspace and are summed in slice order
 *   by a second launch (deterministic): kfac_conv_backward_weight_workspace(c_out, geom,
 *   with_bias) bytes; NULL / 0 runs the whole contraction in one pass per tile (correct, but
 *   few workgroups when c_out and kh kw channels are small and n is large).
 * Errors: KFAC_EINVAL for null required pointers, non-positive sizes, an empty output, a
 * short leading dimension or d != kh kw channels + append_ones; KFAC_EWORKSPACE for a
 * non-null workspace smaller than the query; KFAC_EUNSUPPORTED beyond 32-bit indexing.
 */
typedef struct {
  int64_t batch, height, width, channels;
  int64_t kh, kw, pad, stride;
} kfac_conv_geom;

size_t kfac_conv_ea_update_workspace(int64_t d, const kfac_conv_geom* geom);
kfac_status kfac_conv_ea_update(float* F, int64_t d, int64_t ldf, const uint16_t* x, const kfac_conv_geom* geom,
                                int append_ones, float rho, float scale, uint16_t* F_bf16, int64_t ldfb,
                                void* workspace, size_t ws_bytes, kfac_stream_t stream);
size_t kfac_conv_backward_weight_workspace(int64_t c_out, const kfac_conv_geom* geom, int with_bias);
kfac_status kfac_conv_backward_weight(const uint16_t* g, int64_t c_out, const uint16_t* x,
                                      const kfac_conv_geom* geom, float* dWb, int64_t lddw, int with_bias,
                                      float* Gamma, int64_t ldgam, uint16_t* Gamma_bf16, int64_t ldgb,
                                      float rho, float scale, void* workspace, size_t ws_bytes,
                                      kfac_stream_t stream);

/*
 * Grouped plan -- one K-factor step of a whole network (all factors and layers) as a
 * fixed sequence of grouped launches: every launch covers one phase (EA tiles, sketch
 * GEMM, Gram, Cholesky, eigensolver stage, preconditioner product, ...) of every factor or
 * layer at once, so the many small, latency-bound pieces of different factors run
 * concurrently.  The sequence is stream-ordered and contains no allocation, copy or
 * memset, so it can be captured into a hipGraph once and replayed.  The EA step follows
 * Alg. 1's EA lines, the inversion Alg. 3 (SREVD) and the preconditioner the Sec. 4.1
 * identity used by Alg. 5 -- exactly as kfac_ea_update / kfac_rand_eig /
 * kfac_precondition do one factor or layer at a time.
 *
 * Usage: kfac_plan_create -> kfac_plan_workspace -> (allocate) -> kfac_plan_set_scalars
 * -> kfac_plan_upload (copies the task tables into the workspace; call again after
 * changing scalars, outside any graph capture) -> kfac_plan_launch (capturable, repeatable)
 * -> kfac_plan_destroy.  Limits: l = min(r+p, d) <= 288 for every factor.
 *
 * Ownership: create copies the descriptors; the buffers they point to (F, F_bf16, X, U,
 * D, J, S), the workspace and dev_status belong to the caller and must stay valid while
 * the plan (or a graph holding its launches) is used.  The workspace head holds the task
 * tables written by upload; the rest is scratch.  dev_status receives KFAC_DS_* bits OR-ed
 * over all factors (the caller clears it).  Errors: KFAC_EINVAL for a bad descriptor
 * (bad sizes or strides, a layer whose factor index is out of range, J aliasing S,
 * missing F_bf16 on the bf16 path), KFAC_EUNSUPPORTED for l > 288, KFAC_EWORKSPACE for a
 * short workspace, KFAC_EHIP when a launch or the table copy fails.
 */
typedef struct kfac_plan kfac_plan;

typedef struct {
  float* F; int64_t d, ldf;            /* factor, d x d fp32, symmetric                     */
  uint16_t* F_bf16; int64_t ldfb;      /* bf16 copy of F; required for KFAC_SKETCH_BF16;    */
                                       /* refreshed by the EA phase when X is given          */
  int64_t r, p; int q;                 /* rank, oversampling, power iterations              */
  uint64_t stream_id;                  /* Omega stream (see kfac_gaussian_omega)            */
  const void* X; kfac_dtype xtype;     /* EA input (n x d_in, ldx); X == NULL: no EA update */
  int64_t n, d_in, ldx; int append_ones; float scale;
  float* U; int64_t ldu; float* D;     /* outputs: U d x r, D r                             */
  kfac_variant variant;                /* SREVD (Alg. 3) or RSVD (Alg. 2), see kfac_variant  */
} kfac_factor_desc;

typedef struct {
  int fa, fg;                          /* factor indices of the A (input) and G (output) side */
  const float* J; int64_t ldj;         /* gradient d_g x d_a                                  */
  float* S; int64_t lds;               /* preconditioned gradient d_g x d_a                   */
} kfac_layer_desc;

kfac_status kfac_plan_create(const kfac_factor_desc* factors, int nf, const kfac_layer_desc* layers, int nl,
                             kfac_precision prec, kfac_plan** out);
size_t kfac_plan_workspace(const kfac_plan* plan);
/* Defaults: rho 0.95, lambda 0.1, seed 0, inversion_index 0, all phases on. */
kfac_status kfac_plan_set_scalars(kfac_plan* plan, float rho, float lambda, uint64_t seed,
                                  uint32_t inversion_index, int do_ea, int do_eig, int do_precondition);
kfac_status kfac_plan_upload(kfac_plan* plan, void* workspace, size_t ws_bytes, int32_t* dev_status,
                             kfac_stream_t stream);
/* Number of grouped launches one kfac_plan_launch issues (after upload). */
int kfac_plan_launch_count(const kfac_plan* plan);
/* Enqueue every grouped launch on `stream` (no host synchronisation, no allocation). */
kfac_status kfac_plan_launch(const kfac_plan* plan, kfac_stream_t stream);
/* Enqueue launches [first, first+count) only, in order (for per-phase timing). */
kfac_status kfac_plan_launch_range(const kfac_plan* plan, int first, int count, kfac_stream_t stream);
/* Phase name of launch `index` ("gemm_bf16", "tridiag", ...), NULL when out of range. */
const char* kfac_plan_launch_name(const kfac_plan* plan, int index);
/* Algorithmic work of launch `index`, summed over its tasks: flops of the operation as
 * defined (no padding, no split-K partials) and the minimum bytes it must move (each
 * operand read once, each result written once).  KFAC_EINVAL when out of range. */
kfac_status kfac_plan_launch_work(const kfac_plan* plan, int index, double* flops, double* bytes);
/*
 * Autotuner: for every grouped fp32 GEMM launch of the plan, times each tile configuration
 * (64x64, 128x128, 96x128, 128x64, and 288x64 over the whole sketch width where M <= 288 and
 * no operand is transposed), and for every bf16 sketch / power-iteration launch each
 * kernel (96x128 tiles, or full-sketch-width tiles with split-K and its reduction), over
 * `reps` launches after one warm-up, and keeps the fastest; then uploads the tables again.
 * Results are keyed by a hash of the library's sources and build flags, the device
 * architecture, the HIP runtime version and the launch's shapes (layout and every task's
 * M, N, K), and appended to the text file `cache_path` (nullable), whose entries are
 * reused without timing.  Runs kernels and synchronises the stream: call it
 * after kfac_plan_upload's arguments are final and outside any graph capture.  The tuned
 * launches write only buffers that later launches of the step overwrite (workspace, U, S).
 * With the environment variable KFAC_AUTOTUNE_VERBOSE set (non-zero), every candidate's
 * time is printed to stderr.
 */
kfac_status kfac_plan_autotune(kfac_plan* plan, void* workspace, size_t ws_bytes, int32_t* dev_status,
                               const char* cache_path, int reps, kfac_stream_t stream);
/*
 * Concurrent branches: the plan's layers (each with its two factors) and unused factors are
 * split into nbranch groups (1..4) that run on separate streams: kfac_plan_launch records
 * an event on the caller's stream, makes nbranch - 1 plan-owned streams wait for it,
 * enqueues every group's launches on its own stream (group 0 on the caller's) and joins
 * them back into the caller's stream, so a capture of kfac_plan_launch holds parallel
 * branches.  The layers with the largest EA work form the last group and the rest are
 * balanced over the others, so the latency-bound eigensolver phases of one group (a few
 * workgroups each) overlap the streaming phases of another.  Results are identical to
 * nbranch = 1 (the default).  Streams and events are created here (default priority);
 * takes effect at the next kfac_plan_upload and resets the autotuned configurations.
 * kfac_plan_launch_branch gives the group of launch `index` (-1 out of range; nbranch
 * marks layers preconditioned after the join because their factors sit in two groups).
 */
kfac_status kfac_plan_set_branches(kfac_plan* plan, int nbranch);
int kfac_plan_launch_branch(const kfac_plan* plan, int index);
/* Sets every fp32 GEMM launch to configuration cfg_gemm_f32 (0..4; 4, the whole-sketch-width
 * tile, only where it applies) and every bf16 sketch launch to cfg_sketch_bf16 (0..1); -1
 * keeps the default.  Takes effect at the next kfac_plan_upload.  For tests and experiments. */
kfac_status kfac_plan_force_config(kfac_plan* plan, int cfg_gemm_f32, int cfg_sketch_bf16);
/* Configuration of launch `index` (fp32 GEMM: 0..4; bf16 sketch: 0..1; 0 otherwise; -1 when
 * out of range). */
int kfac_plan_launch_config(const kfac_plan* plan, int index);
void kfac_plan_destroy(kfac_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* KFAC_H */
