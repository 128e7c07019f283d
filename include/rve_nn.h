/* rve_nn.h - C ABI of the learned warm start: kernels of a 3-D convolutional encoder-decoder that
 * predicts the strain fluctuation field of an RVE from its voxel fraction field, trained on fields
 * the Galerkin solver itself produces, with BF16 weights and activations and FP32 accumulation on
 * MFMA (gfx950).
 *
 * The paper solves every RVE from a zero start (Sec. 2, MINRES on the Galerkin system, eq. galres);
 * the network only supplies a starting field, which solve_rve (rve.h) projects onto compatible
 * fields (eq. galop with C = identity) and replaces by zero when its residual is not below the
 * right-hand side.  The converged result is therefore the same fixed point as without it.
 *
 * Conventions shared by every entry point:
 *   - All data pointers are device pointers, owned by the caller, and must stay valid until the
 *     work queued on hip_stream (a hipStream_t, NULL = default stream) has finished; every call
 *     only enqueues work and returns.
 *   - Activations are channels-last BF16 (raw uint16 storage): element (v, c) of a tensor with
 *     channel stride S and channel offset O sits at index v*S + O + c, v the linear voxel index of
 *     dims4 = {batch, n0, n1, n2} (n2 fastest).  Offsets let a layer read or write one channel
 *     slice of a concatenation buffer.
 *   - Convolutions are periodic (circular padding: the RVE is a periodic cell).  Weights are BF16
 *     W[tap][n][k] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1) for ksize 3, tap 0 for ksize 1; n output
 *     channel, k input channel); biases FP32 [n].
 *   - Errors: RVE_EINVAL for a NULL pointer, a bad size, stride, offset or channel count (checked
 *     before any launch, nothing is enqueued); RVE_ENOMEM when a workspace is too small;
 *     RVE_EDEVICE when a launch fails.
 */
#ifndef RVE_NN_H
#define RVE_NN_H

#include <stddef.h>
#include <stdint.h>

#include "rve.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { RVE_NN_POOL2 = 0, RVE_NN_POOL2_BWD_ACC = 1, RVE_NN_UP2 = 2, RVE_NN_UP2_BWD = 3 };

/* 3-D convolution, ksize 1 or 3:
 *   y[v][n] = act(sum_tap sum_k x[v + off(tap)][k] W[tap][n][k] + bias[n]) * (mask[v][n] > 0 if mask)
 * act = ReLU if relu, identity otherwise; bias may be NULL; mask (BF16, stride m_stride, offset
 * m_off) may be NULL.  cin and cout multiples of 16, cout <= 256; x_stride and x_off multiples of 4.
 * y is FP32 if y_f32, else BF16 (rounded to nearest even).
 * The data gradient of a convolution is this call on dy with the weights from rve_nn_flip_weights,
 * with mask = the layer input when that input is a ReLU output. */
rve_status rve_nn_conv3d(const void* x, int32_t cin, int32_t x_stride, int32_t x_off, const void* w, const float* bias,
                         int32_t cout, void* y, int32_t y_stride, int32_t y_off, int32_t y_f32, int32_t relu,
                         const void* mask, int32_t m_stride, int32_t m_off, const int32_t* dims4, int32_t ksize,
                         void* hip_stream);

/* Weight and bias gradients of rve_nn_conv3d (FP32, overwritten):
 *   dw[tap][n][k] = sum_v dy[v][n] x[v + off(tap)][k],   db[n] = sum_v dy[v][n]   (db may be NULL)
 * Summed per voxel chunk on MFMA, then over chunks in a fixed order (deterministic).  workspace:
 * device scratch of at least rve_nn_wgrad_workspace_bytes bytes. */
size_t rve_nn_wgrad_workspace_bytes(int32_t cin, int32_t cout, const int32_t* dims4, int32_t ksize);
rve_status rve_nn_conv3d_wgrad(const void* x, int32_t cin, int32_t x_stride, int32_t x_off, const void* dy,
                               int32_t cout, int32_t dy_stride, int32_t dy_off, float* dw, float* db,
                               const int32_t* dims4, int32_t ksize, void* workspace, size_t workspace_bytes,
                               void* hip_stream);

/* wd[t][k][n] = w[taps-1-t][n][k]: weights (BF16, cin -> cout) of the adjoint convolution
 * (cout -> cin, offsets negated). */
rve_status rve_nn_flip_weights(const void* w, void* wd, int32_t cin, int32_t cout, int32_t ksize, void* hip_stream);

/* Resampling between levels, c channels, BF16:
 *   RVE_NN_POOL2          y = 2x2x2 mean of x                (dims4 = fine dims, all even)
 *   RVE_NN_POOL2_BWD_ACC  y[child] += (mask[child] > 0) x[parent] / 8   (x = coarse gradient,
 *                         y = fine gradient, mask = fine ReLU output; dims4 = fine dims)
 *   RVE_NN_UP2            y[child] = x[parent], nearest      (dims4 = coarse dims)
 *   RVE_NN_UP2_BWD        y[parent] = sum of x over the 8 children (dims4 = coarse dims)
 * mask is used by RVE_NN_POOL2_BWD_ACC only. */
rve_status rve_nn_resample(int32_t op, const void* x, int32_t c, int32_t x_stride, int32_t x_off, void* y,
                           int32_t y_stride, int32_t y_off, const void* mask, int32_t m_stride, int32_t m_off,
                           const int32_t* dims4, void* hip_stream);

/* Network input in BF16: out[v][out_channels] = (phi[v], extra_0[v], ..., extra_{n_extra-1}[v], 0, ...)
 * for n_samples samples of nvox_per_sample voxels; phi FP32 [sample][voxel], extra FP32
 * [sample][n_extra][voxel] (may be NULL when n_extra = 0); out_channels a multiple of 16 and at
 * least 1 + n_extra. */
rve_status rve_nn_pack_input(const float* phi, const float* extra, int32_t n_extra, void* out, int32_t out_channels,
                             int64_t nvox_per_sample, int32_t n_samples, void* hip_stream);

/* Weighted squared error of n_channels predicted fields and its gradient.
 *   pred: FP32 [v][pred_stride] over n_samples samples of nvox_per_sample voxels;
 *   target: FP32 [sample][n_channels][nvox_per_sample] (component-major, as solve_rve writes fields);
 *   weight w(v) = weight3[0] + weight3[1] phi[v] + weight3[2] [0 < phi[v] < 1] (phi FP32
 *   [sample][voxel]; weight3 host float[3]: constant, solid-fraction and partial-voxel terms).
 *   dpred (BF16 [v][dpred_stride]) = 2 w (pred - target) inv_norm for channels < n_channels, 0 above;
 *   partials (device FP64 [n_partials]) = per-block sums of w (pred - target)^2; the loss is
 *   inv_norm * sum(partials). */
rve_status rve_nn_loss(const float* pred, int32_t pred_stride, const float* target, int32_t n_channels,
                       const float* phi, const float* weight3, int64_t nvox_per_sample, int32_t n_samples,
                       float inv_norm, void* dpred, int32_t dpred_stride, double* partials, int32_t n_partials,
                       void* hip_stream);

/* Adam step `step` (>= 1, bias corrections 1 - beta^step) on FP32 master weights p with gradient g
 * and moments m, v (all FP32 [n]); weight_decay adds weight_decay * p to g.  p_bf16 (may be NULL)
 * receives the updated weights rounded to BF16. */
rve_status rve_nn_adam(float* p, const float* g, float* m, float* v, void* p_bf16, int64_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step, float weight_decay, void* hip_stream);

/* b = BF16(a), n elements. */
rve_status rve_nn_to_bf16(const float* a, void* b, int64_t n, void* hip_stream);

/* coarse = mean of phi over factor^3 blocks (one sample, n3 = fine dims, each a multiple of factor). */
rve_status rve_nn_restrict(const float* fine, const int32_t* n3, int32_t factor, float* coarse, void* hip_stream);

/* Starting field on the fine grid from the coarse prediction (FP32 [v][pred_stride], channel 6J + c =
 * component c of the fluctuation for unit Mandel macro strain e_J):
 *   eps[c][v] = sum_J E[J] * trilinear_periodic(pred[.][6J + c])(v),   coarse3 = coarse dims,
 * fine dims = factor * coarse3, coarse voxel centres at (i + 1/2) factor fine voxels.
 * macro_strain_dev: device FP64 [6]; eps: device FP32 [6][N] (the solver's field layout). */
rve_status rve_nn_prolong(const float* pred, int32_t pred_stride, const int32_t* coarse3, int32_t factor,
                          const double* macro_strain_dev, float* eps, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RVE_NN_H */
