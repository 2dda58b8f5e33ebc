/*
 * mcaad_surrogate.h - C ABI of the learned surrogate of the calibration
 * library: a multilayer perceptron theta -> E y (n_in -> H -> H -> H -> n_out,
 * SiLU hidden activations, linear output) that also returns its input
 * Jacobian dE y/dtheta, trained on prices and Jacobians that the Monte Carlo
 * path generates (calibrate_jacobian), with a price + gradient loss.
 *
 * Arithmetic: weights kept in FP32 (master copy, Adam moments) with bf16
 * copies for the matrix products, which run on bf16 MFMA with FP32
 * accumulation; activations are rounded to bf16 where they enter a product;
 * elementwise work (SiLU and its derivatives, tangents, loss, Adam) is FP32;
 * the loss is summed in FP64 in a fixed order.
 *
 * Conventions as in mcaad.h: "d_" = device pointer owned by the caller,
 * stream = hipStream_t as void*, 0 = success, negative = error with
 * mlp_last_error(ctx) describing it, nothing allocated inside a call except
 * in mlp_create.  Calls on one context are serialised by the caller.
 *
 * Parameter packing (FP32): W1 [n_in x H] row-major, b1 [H], W2 [H x H],
 * b2 [H], W3 [H x H], b3 [H], W4 [H x n_out], b4 [n_out].
 * Scaling: the network sees x_j = (theta_j - in_shift_j) * in_scale_j and
 * produces z_i; prices are y_i = z_i * out_scale_i + out_shift_i, so
 * dy_i/dtheta_j = dz_i/dx_j * out_scale_i * in_scale_j.
 */
#ifndef MCAAD_SURROGATE_H
#define MCAAD_SURROGATE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_ctx mlp_ctx;

/* n_in in 1..16, H a multiple of 128 in 128..1024, n_out in 1..64,
 * max_batch in 1..65536 (rounded up to a multiple of 64 internally).
 * Allocates every buffer the other calls use; the scaling starts as the
 * identity and the parameters as zero. */
int mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, mlp_ctx **out);
int mlp_destroy(mlp_ctx *ctx);
int64_t mlp_num_params(const mlp_ctx *ctx);

/* d_params: packed FP32 parameters (see above); resets the Adam moments. */
int mlp_set_params(mlp_ctx *ctx, const float *d_params, void *stream);
int mlp_get_params(const mlp_ctx *ctx, float *d_params, void *stream);

/* Affine input/output scaling (FP32 device arrays of n_in and n_out). */
int mlp_set_scaling(mlp_ctx *ctx, const float *d_in_shift, const float *d_in_scale, const float *d_out_shift,
                    const float *d_out_scale, void *stream);

/* Inference: d_theta [B x n_in] -> d_Y [B x n_out] prices and
 * d_J [B x n_out x n_in], J[b][i][j] = dy_i/dtheta_j.  B in 1..max_batch.
 * Batches of at most 64 samples (with n_in <= 8) run in one launch, one
 * workgroup per sample; larger ones as products over the whole batch.  Both
 * take the same MFMA products of the same bf16 operands in the same order and
 * the same elementwise arithmetic, so a sample's outputs do not depend on the
 * size of the batch it is evaluated in. */
int mlp_forward(mlp_ctx *ctx, const float *d_theta, int32_t B, float *d_Y, float *d_J, void *stream);

/* Loss and its gradient for one batch: with z the network output and zl, jl
 * the labels in network units (zl_i = (y_i - out_shift_i)/out_scale_i,
 * jl_ij = dy_i/dtheta_j / (out_scale_i in_scale_j)),
 *   L = mean_{b,i} (z - zl)^2 + w mean_{b,i,j} c_b (dz_i/dx_j - jl_ij)^2
 * with per-sample weights c_b of the Jacobian term from d_jw [B] (FP32; NULL:
 * all 1): a sample whose Jacobian label is not to be trusted gets 0 and
 * contributes its prices only (its Jacobian label is then never read as a
 * number).  d_idx [B] (int32, may be NULL): sample b of the batch is row
 * d_idx[b] of d_theta, d_Ylab, d_Jlab and d_jw (NULL: row b), so batches can
 * be drawn from a resident data set without gathering them first.
 * Labels are given in price units: d_Ylab [B x n_out], d_Jlab
 * [B x n_out x n_in].  B must be a multiple of 128.  d_loss[1] (FP64) and
 * d_grad [num_params] (FP32, packed like the parameters) are written.
 * For n_in <= 7 the weight and bias gradients of each layer run on a second
 * stream the context owns, forked from `stream` by events as soon as the
 * layer's adjoints exist and joined back to it before the call returns: all
 * the call's work is ordered on `stream` as if it ran there (and the call can
 * be captured into a graph on `stream`); two calls on one context must not
 * overlap. */
int mlp_loss_grad(mlp_ctx *ctx, const float *d_theta, const float *d_Ylab, const float *d_Jlab, const float *d_jw,
                  const int32_t *d_idx, int32_t B, float w, double *d_loss, float *d_grad, void *stream);

/* One Adam step (Kingma & Ba) with bias correction for step t >= 1 on the
 * FP32 master parameters, then refresh of the bf16 copies. */
int mlp_adam_step(mlp_ctx *ctx, const float *d_grad, float lr, float beta1, float beta2, float eps, int32_t t,
                  void *stream);

/* mlp_adam_step with the learning rate d_lr[0] (FP32) and the step count
 * d_t[0] (int32, >= 1) read on the device, and d_t[0] incremented there
 * afterwards: a training loop of such calls, with its batches given by
 * d_idx, launches the same work every epoch and can be captured in a graph
 * and replayed. */
int mlp_adam_step_dev(mlp_ctx *ctx, const float *d_grad, const float *d_lr, float beta1, float beta2, float eps,
                      int32_t *d_t, void *stream);

/* The surrogate's calibration functional (the paper's eq. 241118A with the
 * network's prices in place of the Monte Carlo means): for each of B
 * parameter vectors, d_Y/d_J as in mlp_forward, then in FP64
 * r = y - C, d_G[b] = 1/2 sum_i r_i^2, d_grad[b*n_in + j] = sum_i J_ij r_i.
 * d_C [n_out] FP64 targets. */
int mlp_calibration_gradient(mlp_ctx *ctx, const float *d_theta, int32_t B, const double *d_C, float *d_Y,
                             float *d_J, double *d_G, double *d_grad, void *stream);

const char *mlp_last_error(const mlp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MCAAD_SURROGATE_H */
