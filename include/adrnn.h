/*
 * adrnn.h -- C ABI of the learned warm start for the directional diffusion
 * splitting solver (gfx950, BF16 matrix cores with FP32 accumulation).
 *
 * The network predicts the stationary solution of eq. (1) from the problem
 * data, as a correction to the initial iterate of eq. (11) (the s-solve on the
 * beta-curves).  The splitting method then iterates from that prediction and
 * remains the judge of the result (adr_split_iterate's residual).
 *
 * Network: four 3x3 convolutions with zero padding, 4 -> 32 -> 32 -> 32 -> 1
 * channels, dilations 1, 2, 4, 8 (tap (dy, dx) of layer l reads the pixel
 * d_l (dy, dx) away; a 31 x 31 receptive field), ReLU after the first three.  Tensors are NHWC over B images of
 * H x W pixels (pixel p = y*W + x, the solver's grid layout).  Stored
 * activations and matrix-core operands are BF16 (round to nearest even);
 * products accumulate in FP32; master weights, Adam moments, biases, the
 * output and the loss gradient are FP32.
 *
 * Parameter vector (FP32, adrnn_param_count() = 19969 entries):
 *   W1[32][3][3][4], b1[32], W2[32][3][3][32], b2[32], W3[32][3][3][32], b3[32],
 *   W4[1][3][3][32], b4[1]      (W[n][dy+1][dx+1][c], tap (dy,dx))
 *
 * Inputs (adrnn_pack): channel 0 = f / |f|_inf, 1 = log10(mu) + 2,
 * 2 = s / |s|_inf (s = eq. (11) iterate), 3 = interior mask.
 * Target (training): (u* - s) / |s|_inf on interior pixels, u* the converged
 * solution.  Prediction (adrnn_warm_start): u = s + |s|_inf * out on interior
 * pixels, 0 elsewhere.  Loss: mean of (out - target)^2 over interior pixels.
 *
 * Memory: all data pointers are device memory owned by the caller unless
 * noted "host".  Work runs on the stream given at creation.  Errors are
 * returned as adr_status codes (ADR_EINVAL, ADR_ENOMEM, ADR_EDEVICE).
 */
#ifndef ADRNN_H
#define ADRNN_H

#include <stdint.h>

#include "adr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adrnn_ctx adrnn_ctx;

int64_t adrnn_param_count(void);

/* Context for images of H x W pixels and batches of at most max_batch images;
 * allocates the activation buffers.  stream: hipStream_t or NULL. */
adr_status adrnn_create(int32_t H, int32_t W, int32_t max_batch, void *stream, adrnn_ctx **out);
adr_status adrnn_destroy(adrnn_ctx *ctx);

/* Copy the FP32 parameter vector in (host) / out (host).  Setting resets the
 * Adam moments and step count. */
adr_status adrnn_set_params(adrnn_ctx *ctx, const float *params);
adr_status adrnn_get_params(adrnn_ctx *ctx, float *params);

/* Build the BF16 input tensor x0 (B*H*W*4) and, when u_star != NULL, the FP32
 * target (B*H*W).  f, s, u_star: FP64 grids (B*H*W); mask: uint8 (H*W, shared
 * by all images); mu: host array of B values.  s_norm (B, FP64, may be NULL)
 * receives |s|_inf per image. */
adr_status adrnn_pack(adrnn_ctx *ctx, int32_t B, const double *f, const double *s, const uint8_t *mask,
                      const double *mu, const double *u_star, void *x0, float *target, double *s_norm);

/* out (FP32, B*H*W) = network(x0). */
adr_status adrnn_forward(adrnn_ctx *ctx, int32_t B, const void *x0, float *out);

/* Loss and its gradient (FP32, parameter layout) for a batch: forward, loss,
 * backward.  grads: device, adrnn_param_count() floats.  The loss is also
 * added to the context's device-side sum (adrnn_loss_sum).  loss (host, may be
 * NULL): this batch's loss; non-NULL synchronises the stream, NULL leaves the
 * call asynchronous. */
adr_status adrnn_grads(adrnn_ctx *ctx, int32_t B, const void *x0, const float *target, const uint8_t *mask,
                       float *grads, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the device master weights. */
adr_status adrnn_adam(adrnn_ctx *ctx, const float *grads, float lr);

/* Sum (host, may be NULL) and count (host, may be NULL) of the losses of the
 * adrnn_grads / adrnn_train_step calls since the context was created or last
 * reset; reset != 0 clears both afterwards.  Synchronises the stream. */
adr_status adrnn_loss_sum(adrnn_ctx *ctx, double *sum, int64_t *steps, int32_t reset);

/* adrnn_grads followed by adrnn_adam with the context's gradient buffer. */
adr_status adrnn_train_step(adrnn_ctx *ctx, int32_t B, const void *x0, const float *target, const uint8_t *mask,
                            float lr, double *loss);

/* u (FP64 grids, B*H*W) = s + |s|_inf * out on interior pixels, 0 elsewhere.
 * s_norm: device FP64 (B) from adrnn_pack. */
adr_status adrnn_warm_start(adrnn_ctx *ctx, int32_t B, const double *s, const double *s_norm, const float *out,
                            const uint8_t *mask, double *u);

/* Coarse-grid use of the network.  The context's H x W pixels are then the
 * nodes of a coarse grid inside a fine grid of Hf = r (H - 1) + 1 by
 * Wf = r (W - 1) + 1 nodes (integer factor r >= 1), coarse node (i, j) lying
 * on fine node (r i, r j); the network sees the problem on the coarse grid,
 * where its 31 x 31 receptive field spans 31 r fine nodes.  Not in the paper:
 * the grid transfers of the multigrid literature (full weighting, bilinear
 * interpolation).
 *
 * adrnn_restrict: coarse (FP64, B*H*W) = R fine (FP64, B*Hf*Wf).  At interior
 * coarse nodes R is the tent-weighted mean of the (2r - 1)^2 fine nodes
 * around the coincident fine node, weight (r - |dy|)(r - |dx|) / r^4; boundary
 * coarse nodes take the coincident fine value.  r = 1 copies.  EINVAL when
 * Wf > 8192 or B*Hf*Wf > 2^31. */
adr_status adrnn_restrict(adrnn_ctx *ctx, int32_t B, int32_t r, const double *fine, double *coarse);

/* adrnn_warm_start for a network run on the coarse grid: u (FP64, B*Hf*Wf) =
 * s + |s|_inf * (P out) on the fine pixels where mask (uint8, Hf*Wf) is set,
 * 0 elsewhere, P the bilinear interpolation of out (FP32, B*H*W, coarse) at
 * the fine nodes, evaluated in FP64:
 *   (P out)(r i + a, r j + c) = [(r-a)(r-c) o(i,j) + (r-a) c o(i,j+1)
 *                                + a (r-c) o(i+1,j) + a c o(i+1,j+1)] / r^2.
 * s, s_norm as in adrnn_warm_start (s_norm from adrnn_pack on the restricted
 * s).  r = 1 gives adrnn_warm_start.  EINVAL when B*Hf*Wf > 2^31. */
adr_status adrnn_warm_start_prolong(adrnn_ctx *ctx, int32_t B, int32_t r, const double *s, const double *s_norm,
                                    const float *out, const uint8_t *mask, double *u);

/* Test export: D (16x16 FP32, row-major) = A (16x16 BF16, row-major) * B
 * (16x16 BF16, row-major) on one wavefront through the same matrix-core
 * instruction and operand layout the convolutions use. */
adr_status adrnn_mfma_probe(const void *A, const void *B, float *D, void *stream);

const char *adrnn_last_error(const adrnn_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADRNN_H */
