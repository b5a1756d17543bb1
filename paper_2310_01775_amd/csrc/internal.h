// Host-side launchers of the STAMP kernels (internal to libstamp.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace stamp {

// packed: one lane per (particle, side) holding all B blocks, instead of one
// lane per block (same results bit for bit, same tape layout).
hipError_t launch_rollout_fwd(const SimConst& c, int N, const float* theta, float* cost, float* tape,
                              const TapeGeom& g, uint32_t* status, hipStream_t st, bool packed);
hipError_t launch_rollout_adj(const SimConst& c, int N, const float* theta, const float* tape,
                              const TapeGeom& g, const float* cost_bar, float cb_scalar, float* grad,
                              float* seg, uint32_t* status, hipStream_t st, bool packed);

// Particles per 64-lane rollout tile of a problem with B blocks.
int rollout_tile_particles(int B, bool packed);
hipError_t launch_rollout_fwd_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, float* cost, float* tape, uint32_t* status,
                                      hipStream_t st, bool packed);
hipError_t launch_rollout_adj_batched(const ProblemDesc* descs, const int2* tiles, int ntiles, int block,
                                      int grid, const float* theta, const float* tape, float cb_scalar,
                                      float* grad, float* seg, uint32_t* status, hipStream_t st, bool packed);

// SVGD step of one problem.  h: when bandwidth > 0 it is used as is; otherwise
// the median heuristic runs and writes h into the workspace (and h_out if
// non-null).  phi_rows: rows per contraction workgroup (0 = 256).
SvgdLayout svgd_workspace_layout(int N, int d);
// class index (0 .. kPhi32Classes-1) of the FP32 direction's contraction for dimension d
// (0, 1: the split form for d <= kPhi3MaxD; then the FP32 matrix-core form)
int phi32_class(int d);
// wts: null, or per-particle importance weights (mean 1) of Eq. (4).
hipError_t launch_svgd(int N, int d, const float* theta, const float* grad_logp, float bandwidth, float* phi,
                       float* h_out, void* ws, const SvgdLayout& L, int phi_rows, uint32_t* status,
                       hipStream_t st, const float* wts = nullptr);
// The step's first half, which depends on theta only (and may therefore run
// concurrently with the rollout that produces grad_logp): the median into the
// workspace's selection state and the FP32 form's theta operands (particle
// mean, centred rows, norms -- which the median's Gram-form passes read).
hipError_t launch_svgd_bandwidth(int N, int d, const float* theta, float bandwidth, float* h_out, void* ws,
                                 const SvgdLayout& L, hipStream_t st);
// step (nullable): advanced once by the stage's first launch (only when
// P.n_ctr > 0: some problem has N >= 2)
hipError_t launch_svgd_bandwidth_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, int exact,
                                         char* ws, hipStream_t st, int* step = nullptr);
// particle mean, centred rows and norms (before the median)
hipError_t launch_operands32(int N, int d, const float* theta, void* ws, const SvgdLayout& L, hipStream_t st);
hipError_t launch_operands32_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws,
                                     hipStream_t st, int* step = nullptr);
// The step's second half: V = w [g - (2/h) x | 1] packed from theta, the
// gradient and the weights, then phi from the bandwidth, centre and rows the
// workspace holds (FP32 matrix cores, phi32.hip).
// upd (nullable): apply the update of Algorithm 1 to theta in the same pass
// (phi may then be null); theta is read for every element before its update.
hipError_t launch_svgd_direction(int N, int d, const float* theta, const float* grad_logp, float* phi, void* ws,
                                 const SvgdLayout& L, int phi_rows, uint32_t* status, hipStream_t st,
                                 const float* wts = nullptr, const UpdateArgs* upd = nullptr);
hipError_t launch_svgd_direction_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta,
                                         const float* grad, float* phi, char* ws, uint32_t* status, hipStream_t st,
                                         const float* wts = nullptr, const UpdateArgs* upd = nullptr);
// The same step for every problem of a batch (work lists in P); wts packed
// like the costs (problem p at its cost offset), or null.
hipError_t launch_svgd_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, const float* grad,
                               float* phi, char* ws, uint32_t* status, hipStream_t st, const float* wts = nullptr);
// phi = (sum over the splits of partial[q][d][N], in split order) / N.
hipError_t launch_phi_reduce(int N, int d, int splits, const float* partial, float* phi, uint32_t* status,
                             hipStream_t st);
// SVGD step under the structured pusher kernel (structured.hip); wts null or
// importance weights; h_out (nullable) receives (h_g, h_z).
hipError_t launch_svgd_structured(int N, int d, const float* theta, const float* grad, const float* wts,
                                  const StructKernel& sk, float* phi, float* h_out, void* ws, const SvgdLayout& L,
                                  uint32_t* status, hipStream_t st);
// its two halves: features + medians (theta only), then the contraction
hipError_t launch_struct_bandwidth(int N, const float* theta, const StructKernel& sk, void* ws, const SvgdLayout& L,
                                   hipStream_t st);
hipError_t launch_struct_direction(int N, int d, const float* grad, const float* wts, const StructKernel& sk,
                                   float* phi, float* h_out, void* ws, const SvgdLayout& L, uint32_t* status,
                                   hipStream_t st);
// Importance weights of Eq. (4): w_j = N softmax_j(C_disc - C_rel), mean 1.
hipError_t launch_dsvgd_weights(int N, const float* c_rel, const float* c_disc, float* w, hipStream_t st);
hipError_t launch_dsvgd_weights_batched(int n_problems, const ProblemDesc* descs, const float* c_rel,
                                        const float* c_disc, float* w, hipStream_t st);

// Median-heuristic bandwidth into the problem's SelState (median.hip): exact = 1
// the exact lower median of all pairs, 0 the lower median of a fixed sample.
// gram = 1: problems above 2^20 pairs take, in their passes over every pair,
// the Gram-form distances of the FP32 contraction's operands (which the
// workspace must already hold for this theta: launch_operands32); smaller ones
// keep direct differences.  The batched median always does so: its work lists
// fix each problem's form (exact = 1 needs the operands of the large ones).
hipError_t launch_median(int N, int d, const float* theta, float bandwidth, int exact, void* ws, const SvgdLayout& L,
                         float* h_out, hipStream_t st, int gram = 0);
hipError_t launch_median_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, int exact,
                                 char* ws, hipStream_t st);

// The same step on the BF16 matrix cores with a sampled median (phi16.hip).
hipError_t launch_svgd16(int N, int d, const float* theta, const float* grad, float bandwidth, float* phi,
                         float* h_out, void* ws, const SvgdLayout& L, uint32_t* status, hipStream_t st);
hipError_t launch_svgd16_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, const float* grad,
                                 float* phi, char* ws, uint32_t* status, hipStream_t st);
// its theta-only operand (the particle mean), built with the sampled median,
// and its second half (the scaled BF16 rows and V, which need h, the
// contraction, the reduce; upd as for the FP32 form)
hipError_t launch_operands16(int N, int d, const float* theta, void* ws, const SvgdLayout& L, hipStream_t st);
// the sampled median and the centres for a batch, in two launches (sample
// distances with the centres, then the sample select); a non-null step
// counter is advanced by one on the way
hipError_t launch_bandwidth16_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws,
                                      hipStream_t st, int* step = nullptr);
hipError_t launch_svgd16_direction(int N, int d, const float* theta, const float* grad, float* phi, void* ws,
                                   const SvgdLayout& L, uint32_t* status, hipStream_t st,
                                   const UpdateArgs* upd = nullptr);
hipError_t launch_svgd16_direction_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta,
                                           const float* grad, float* phi, char* ws, uint32_t* status,
                                           hipStream_t st, const UpdateArgs* upd = nullptr);

// Adam (use_adam=1) or plain step, n elements.  t_dev: if non-null, the step
// count is read as t0 + *t_dev + 1 on the device (graph replay); else t0 is t.
hipError_t launch_update(int64_t n, float* theta, const float* phi, float* m, float* v, int t0,
                         const int* t_dev, float lr, float b1, float b2, float eps, int use_adam,
                         hipStream_t st);

// Final read-out: Gamma(a_k) = first argmax side per push, modes [H][N].
hipError_t launch_modes(int N, int H, const float* theta, int32_t* modes, hipStream_t st);

// tiny device helpers
hipError_t launch_onehot(int N, int H, const float* theta, float* out, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_incr(int* p, hipStream_t st);

// Surrogate network.  Wb holds the BF16 copies (kMlpBfTotal elements).
struct MlpTrainLayout {
    size_t ut, h1t, d2t, d1t, dw1, dw2, part, total;  // byte offsets into the workspace
};
MlpTrainLayout mlp_train_layout(int M);
hipError_t launch_mlp_prepare(const float* P, __bf16* Wb, hipStream_t st);
// x_mode 0: X is [M][n_in]; x_mode 1: X is [d][M] (structure of arrays) and
// inputs d..n_in-1 are enc[0..n_in-d).  Any of y_out / cost_out / grad_out may
// be null; grad_out is [d][M] = grad_scale * dC_hat/dx.
// bound_H > 0 adds the exact bound term (weight wb) of the first 6*bound_H
// inputs to cost_out and grad_out.
hipError_t launch_mlp_infer(const float* P, const __bf16* Wb, const float* X, int x_mode, int M, int n_in, int d,
                            const float* enc, int bound_H, float wb, float omax, float dmax, float* y_out,
                            float* cost_out, float* grad_out, float grad_scale, hipStream_t st);
// One Adam step of the mean squared error of y against log(1 + cost) over M
// samples (M % 64 == 0), sample i = dataset row idx[i] (or i).
hipError_t launch_mlp_train_step(float* P, __bf16* Wb, float* mom, float* vel, int t, float lr, float b1, float b2,
                                 float eps, const float* X, const float* cost, const int* idx, int n_rows, int M,
                                 int n_in, float* loss_out, uint32_t* status, char* ws, const MlpTrainLayout& L,
                                 hipStream_t st);
// out[p] = mean over problem p's particles of |log(1 + c_sur) - log(1 + c_true)|
// (costs at the problems' cost offsets).
hipError_t launch_log_err(const ProblemDesc* descs, int n_problems, const float* c_true, const float* c_sur,
                          float* out, hipStream_t st);
hipError_t launch_mlp_standardize(const float* X, const float* cost, int M, int n_in, float* P, hipStream_t st);
hipError_t launch_mlp_pack_rows(const float* theta, int N, int d, const float* enc, int n_in, float* Xo,
                                hipStream_t st);

}  // namespace stamp
