// Launch interface between the C ABI (kfac_abi.hip) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>
#include "../../include/kfac.h"
#include "common.h"
#include "gemm_f32.h"
#include "tasks.h"
#include "ea_tile.h"

namespace kfac {

// fp32 kernels (kernels_f32.hip)
hipError_t launch_fill_identity(float* F, int d, long ldf, hipStream_t s);
hipError_t launch_gemm(const GemmP& p, bool ta, bool tb, hipStream_t s);
// EA tiles are 64 x 64 (fp32 MFMA) for fp32 activations and 128 x 128 (bf16 MFMA) for
// bf16 activations; `bf` selects the variant.
int ea_tiles_per_side(int d, bool bf);
int ea_choose_ksplit(int d, long n, bool bf);
size_t ea_workspace_bytes(int d, long n, bool bf);
size_t ea_partial_bytes(int d, int ks, bool bf);   // split-K partial sums of ks slices
// split-K count of one factor inside a grouped EA launch whose factors together take
// total_steps block steps (tiles x 64-row / 32-row steps) without splitting
int ea_grouped_ksplit(int d, long n, bool bf, double total_steps);
size_t ea_workspace_bytes(int d, long n);   // enough for either variant
int ea_finalize_chunks(bool bf);             // finalize blocks per tile
hipError_t launch_ea_f32(float* F, int d, long ldf, const float* X, int n, int d_in, long ldx, int ones,
                         float rho, float scale, uint16_t* Fb, long ldfb, void* ws, size_t ws_bytes,
                         hipStream_t s);
hipError_t launch_ea_bf16(float* F, int d, long ldf, const uint16_t* X, int n, int d_in, long ldx, int ones,
                          float rho, float scale, uint16_t* Fb, long ldfb, void* ws, size_t ws_bytes,
                          hipStream_t s);
hipError_t launch_omega(int d, int l, int d_pad, int l_pad, uint64_t seed, uint64_t stream_id, uint32_t inv,
                        float* OmT, long ldt, uint16_t* OmTb, float* Om, long ldo, uint32_t* words,
                        hipStream_t s);
int sign_chunks(int d);
hipError_t launch_sign_normalize(float* U, long ldu, int d, int r, float* pval, int* pidx, hipStream_t s);

// bf16 sketch GEMM (kernels_bf16.hip): Ct[M x N] = A[M x K] * B[N x K]^T, both K-contiguous
hipError_t launch_gemm_bf16_nt(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb,
                               float* C, long ldc, hipStream_t s);

// K-FAC linear layer (kernels_linear.hip)
hipError_t launch_linear_forward(const uint16_t* x, int n, int d_in, long ldx, const uint16_t* W, int d_out, long ldw,
                                 const float* bias, uint16_t* y, long ldy, hipStream_t s);
hipError_t launch_linear_backward(const uint16_t* g, int n, int d_out, long ldg, const uint16_t* x, int d_in, long ldx,
                                  const uint16_t* W, long ldw, uint16_t* dx, long lddx, float* dWb, long lddw,
                                  int with_bias, float* Gam, long ldgam, uint16_t* Gamb, long ldgb, float rho,
                                  float scale, hipStream_t s);

// fp64 kernels (kernels_f64.hip)
int gram_ksplit(int L, int K, int sym);
size_t gram_workspace_bytes(int L, int K, int sym);
hipError_t launch_gram(const float* A, long lda, const float* B, long ldb, int L, int K, int sym,
                       double* part, double* C, long ldc, int* status, hipStream_t s);
hipError_t launch_cholesky(const double* G, long ldg, int n, long m_rows, double* W, long ldw, double* Li,
                           int* status, int* fail_flag, hipStream_t s);
constexpr int kCholInvMax = 288;   // blocked Cholesky-inverse path handles l_pad <= this
// Second pass of CholeskyQR2 (skip != null): the pass is kept out (*skip = 1, Q copied by
// launch_trmm) when the Gram of the first pass's basis is within kQrKeepTol of I.
constexpr double kQrKeepTol = 5.9604644775390625e-08;   // 2^-24
hipError_t launch_cholinv(double* G, long ldg, int n, long m_rows, double* Linv, long ldl, int l_pad, double* dsave,
                          int* status, int* fail_flag, hipStream_t s, int* skip = nullptr, double tol = 0.0);
hipError_t launch_trmm(const double* Li, long ldl, int n, const float* Yt, long ldy, int ncols, float* Qt, long ldq,
                       uint16_t* Qtb, long ldqb, int l_pad, hipStream_t s, const int* skip = nullptr);
hipError_t launch_trsm(const double* W, long ldw, const double* Li, int n, int l_pad, const float* Yt,
                       long ldy, int ncols, float* Qt, long ldq, uint16_t* Qtb, long ldqb, hipStream_t s);
size_t small_eig_scratch_doubles(int n, int r);
hipError_t launch_small_eig(const double* C, long ldc, const float* Cf, long ldcf, int n, int n_pad, int r,
                            double* A, double* V, double* diag, double* off, double* Z, double* scratch,
                            float* P, long ldp, float* D, double* Dd, int* status, hipStream_t s,
                            int svd = 0);


// ---- grouped launches (one launch covers one phase of many tasks) -----------------------
constexpr int kPlanMaxSketch = 288;   // grouped eigensolver phases use the on-chip kernels
EaTask make_ea_task(float* F, int d, long ldf, const float* X, const uint16_t* Xb, int n, int d_in, long ldx, int ones,
                    float rho, float scale, uint16_t* Fb, long ldfb, float* part, int ks);
OmegaTask make_omega_task(int d, int l, int d_pad, int l_pad, uint64_t seed, uint64_t stream_id, uint32_t inv,
                          float* OmT, long ldt, uint16_t* OmTb, float* Om, long ldo, uint32_t* words);
dim3 omega_grid(const OmegaTask& p);
BfGemmTask make_bf16_task(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb, float* C,
                          long ldc);
int bf16_task_blocks(const BfGemmTask& q);
// skinny sketch GEMM (M <= 288): grouped launch + split-K reduction
int skinny_ksplit(int N, int K);
SkinnyTask make_skinny_task(int M, int N, int K, const uint16_t* A, long lda, const uint16_t* B, long ldb, float* C,
                            long ldc, float* part, int ksplit);
int skinny_blocks(const SkinnyTask& q);
size_t skinny_part_bytes(int M, int N, int K);
hipError_t launch_skinny_g(const SkinnyTask* t, GroupMap gm, int blocks, hipStream_t s);
constexpr int kWholeWidthMaxM = 288;   // rows held by the whole-width (skinny / split) kernels
// split-bf16 product of fp32 operands (hi*hi + hi*lo + lo*hi), same whole-width layout
int split_ksplit(int N, int K);
SplitTask make_split_task(int M, int N, int K, const float* A, long lda, const float* B, long ldb, float* C,
                          long ldc, float* part, int ksplit);
int split_blocks(const SplitTask& q);
size_t split_part_bytes(int M, int N, int K);
hipError_t launch_split_g(const SplitTask* t, GroupMap gm, int blocks, hipStream_t s);
// K-slice reduction shared by both
ReduceTask make_reduce_task(int M, int N, const float* part, float* C, long ldc, int ksplit);
int reduce_blocks(const ReduceTask& q);
hipError_t launch_reduce_g(const ReduceTask* t, GroupMap gm, int blocks, hipStream_t s);
// single-factor forms (one group of one task)
hipError_t launch_skinny(const SkinnyTask& q, hipStream_t s);
hipError_t launch_split(const SplitTask& q, hipStream_t s);
GramP make_gram_task(const float* A, long lda, const float* B, long ldb, int L, int K, int sym, double* part,
                     double* C, long ldc, int* status);
int gram_tiles(int L, int sym);
int gram_reduce_slices();
int trmm_blocks_x(int ncols);
int trmm_blocks_y(int l_pad);
EigTask make_eig_task(const double* C, long ldc, const float* Cf, long ldcf, int n, int n_pad, int r, double* A,
                      double* V, double* diag, double* off, double* Z, double* scratch, float* P, long ldp, float* D,
                      double* Dd, int* status);
int tri_bisect_blocks(int n);
int tri_vec_blocks(int r);
int backtransform_blocks(int r);   // 32 columns per workgroup
// grouped fp32 GEMM tiles: 64x64, 128x128, 96x128, 128x64, and 288x64 "skinny" (whole
// sketch width, no transposes, M <= 288)
constexpr int kGemmConfigs = 5;
int gemm_g_blocks_x(const GemmP& p, int cfg);
int gemm_g_blocks_y(const GemmP& p, int cfg);
int gemm_slice_blocks(const GemmP& p);                // split-K finish blocks (0 if ksplit <= 1)
hipError_t launch_gemm_slices_g(const GemmP* t, GroupMap gm, int blocks, hipStream_t s);
// K slices of the precondition's T1 = J U_a diag(f_a) product
int precondition_ksplit(int64_t d_g, int64_t d_a, int64_t r_a);

hipError_t launch_ea_tiles_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_ea_finalize_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s);
constexpr int kEaBf16Tile = 128;
hipError_t launch_ea_bf16_tiles(const EaTask& q, int tiles, int ks, hipStream_t s);
hipError_t launch_ea_bf16_finalize(const EaTask& q, int tiles, hipStream_t s);
hipError_t launch_ea_bf16_tiles_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_ea_bf16_finalize_g(const EaTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_omega_g(const OmegaTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_sign_partial_g(const SignTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_sign_apply_g(const SignTask* t, GroupMap gm, int blocks, hipStream_t s);
// split: the launch holds split-K tasks (ksplit > 1; no transposes, cfg != 4)
hipError_t launch_gemm_g(const GemmP* t, GroupMap gm, int blocks, bool ta, bool tb, int cfg, bool split, hipStream_t s);
// EA update of a convolution's input factor from the im2col patches of NHWC bf16 input x
hipError_t launch_im2col_stage(const uint16_t* x, const ConvGeom& g, uint16_t* P, int ldp, int n, hipStream_t s);
hipError_t launch_ea_bf16_conv(float* F, int d, long ldf, const uint16_t* x, const ConvGeom& cv, int ones, float rho,
                               float scale, uint16_t* Fb, long ldfb, void* ws, size_t ws_bytes, hipStream_t s);
// weight gradient [dW | db] = g^T [P | 1] of a convolution (P: im2col patches of x), with the
// backward-factor EA of g fused (Gam nullable); split over K slices into ws when given
hipError_t launch_conv_backward_weight(const uint16_t* g, const uint16_t* x, const ConvGeom& cv, int c_out,
                                       float* dWb, long lddw, int with_bias, float* Gam, long ldgam, uint16_t* Gamb,
                                       long ldgb, float rho, float scale, void* ws, size_t ws_bytes, hipStream_t s);
size_t conv_backward_weight_ws_bytes(int c_out, long n, int N);
hipError_t launch_gemm_bf16_g(const BfGemmTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_gram_partial_g(const GramP* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_gram_reduce_g(const GramP* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_cholinv_g(const CholInvTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_trtri_cols_g(const CholInvTask* t, GroupMap gm, int blocks, hipStream_t s);
int trtri_col_blocks(int l_pad);
hipError_t launch_trmm_g(const TrmmTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tridiag_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_prep_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_bisect_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_select_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_vec_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_cluster_lead_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_tri_cluster_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);
hipError_t launch_backtransform_g(const EigTask* t, GroupMap gm, int blocks, hipStream_t s);

}  // namespace kfac
