/* tomo_nn.h — learned start for the accelerated iteration: a 2D U-Net trained and run on
 * the GPU (bfloat16 matrix-core kernels for gfx950, float32 accumulation and master
 * weights), part of libtomo.so.
 *
 * The paper starts the iteration from a ramp-filtered back-projection (Sec. 2.2, Eqs.
 * 12-14) and counts a better start as saved iterations (Sec. 3.2).  This network maps the
 * FBP image to a start closer to the converged reconstruction; tomo_reconstruct runs it
 * with TOMO_INIT_LEARNED (keeping the FBP start where the network's start has the larger
 * objective, or outside the training domain), or takes its output through TOMO_INIT_USER.
 *
 * Network (levels L, base channels C; level l has C 2^l channels at H/2^l x W/2^l):
 *   u = fbp / scale;  E0a = relu(conv(u)), E0 = relu(conv(E0a));
 *   l >= 1: P_l = avgpool2(E_{l-1}), E_la = relu(conv(P_l)), E_l = relu(conv(E_la));
 *   l = L-2..0: D_{L-1} = E_{L-1}; cat_l = [up2(D_{l+1}), E_l] (upsampled channels first),
 *   D_la = relu(conv(cat_l)), D_l = relu(conv(D_la));
 *   r = 1x1 conv of D_0 (C -> 1) + bias;  x0 = fbp + scale * r.
 * conv: 3x3, zero padding, with bias; avgpool2: mean of 2x2 blocks; up2: nearest.
 * Loss: mean over pixels of (r - (target - fbp)/scale)^2.  Optimiser: Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Parameter vector (float32, device): for each 3x3 conv in the order E0a, E0b, E1a, E1b,
 * ..., E(L-1)b, D(L-2)a, D(L-2)b, ..., D0a, D0b: weights [Cout][3][3][Cin] then bias
 * [Cout]; then the head weights [C] and bias [1].
 *
 * Arithmetic: the first conv (one input channel) and the head run in float32; every other
 * conv multiplies bfloat16 weights and activations on the matrix cores with float32
 * accumulation; activations and activation gradients are stored in bfloat16 (rounded to
 * nearest even); weight gradients, parameters and Adam moments are float32.
 *
 * Images and all arrays are device memory; images are [batch][H][W] float32 row-major.
 * Everything is enqueued on the stream given at creation.  Errors are status codes
 * (tomo_status of tomo.h); tomo_unet_last_error gives the message.
 */
#ifndef TOMO_NN_H
#define TOMO_NN_H

#include <stddef.h>
#include <stdint.h>

#include "tomo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomo_unet_s* tomo_unet;

/* Create a network for images of height x width (multiples of 2^(levels-1), at most 32767)
 * and batches up to max_batch.  levels 1..6; base_channels a multiple of 32, at most 256, with
 * base_channels 2^(levels-1) <= 1024.  Errors: INVALID_ARG, NO_DEVICE. */
tomo_status tomo_unet_create(int32_t levels, int32_t base_channels, int32_t max_batch,
                             int32_t height, int32_t width, void* hip_stream, tomo_unet* out);
/* Bytes of device workspace (parameters, Adam moments, gradients, activations). */
tomo_status tomo_unet_workspace_size(tomo_unet net, size_t* bytes);
/* Attach caller-owned device memory (256-byte aligned, >= workspace size); parameters must
 * be set again afterwards.  Errors: INVALID_ARG, WORKSPACE_TOO_SMALL. */
tomo_status tomo_unet_set_workspace(tomo_unet net, void* dev, size_t bytes);
/* Number of float32 parameters. */
tomo_status tomo_unet_num_params(tomo_unet net, int64_t* n);
/* Copy the parameter vector (device float32 [n]) in; resets the Adam moments and step.
 * Errors: NO_WORKSPACE, INVALID_ARG, HIP. */
tomo_status tomo_unet_set_params(tomo_unet net, const float* theta);
/* Copy the current parameter vector out (device float32 [n]).  Errors: NOT_READY. */
tomo_status tomo_unet_get_params(tomo_unet net, float* theta);
/* x0 = fbp + scale * r for a batch (1..max_batch) of FBP images.  scale > 0 (e.g. the RMS of
 * the training FBP images).  Errors: NOT_READY (no parameters), INVALID_ARG, HIP. */
tomo_status tomo_unet_forward(tomo_unet net, const float* fbp, float* x0, int32_t batch,
                              float scale);
/* Forward and backward without an update: loss (device float64, nullable) and the gradient
 * of the loss with respect to the parameter vector (device float32 [n], nullable). */
tomo_status tomo_unet_loss_grad(tomo_unet net, const float* fbp, const float* target,
                                int32_t batch, float scale, float* grad, double* loss);
/* One Adam step on a batch with learning rate lr; loss of the batch before the step into
 * loss (device float64, nullable). */
tomo_status tomo_unet_train_step(tomo_unet net, const float* fbp, const float* target,
                                 int32_t batch, float scale, float lr, double* loss);
/* Training domain of a network: the problems whose reconstructions it was trained on.
 * tomo_reconstruct with TOMO_INIT_LEARNED uses the network only on a coarsest level with
 * N_0 == n (== height == width of the network), n_det_0 == n_det, centre c_0 within 1e-6 of
 * center (NaN -> n_det / 2), n_angles_min <= n_angles <= n_angles_max, and the same prior
 * (beta, p, sigma, T within a relative 1e-9, the same neighbourhood). */
typedef struct {
  int32_t n, n_det;
  int32_t n_angles_min, n_angles_max;
  double center;
  double beta, p, sigma, T;
  int32_t neighbours;
} tomo_unet_domain_t;
/* Record (domain != NULL) or clear (NULL) the training domain.  Errors: INVALID_ARG. */
tomo_status tomo_unet_set_domain(tomo_unet net, const tomo_unet_domain_t* domain);
tomo_status tomo_unet_destroy(tomo_unet net);
const char* tomo_unet_last_error(tomo_unet net);

/* Layer-level entry points (bfloat16 arrays as uint16_t; NHWC [batch][H][W][ld], the tensor
 * occupying channels 0..C-1 from the given pointer, 16-byte aligned; cin, cout multiples of
 * 32; ld multiples of 8; H and W at most 32767).
 * tomo_nn_conv3x3: y = relu(bias + conv(x, w)) (relu = 1, bias required), or
 * y = bias + conv(x, w) (bias nullable), optionally times (mask > 0) (mask: bfloat16 with
 * channel count cout and stride ldm; no bias then).  w: bfloat16 [cout][3][3][cin].
 * Output rounded to bfloat16.  Errors: INVALID_ARG, HIP. */
tomo_status tomo_nn_conv3x3(const uint16_t* x, int32_t ldx, const uint16_t* w, const float* bias,
                            uint16_t* y, int32_t ldy, const uint16_t* mask, int32_t ldm,
                            int32_t cin, int32_t cout, int32_t batch, int32_t height,
                            int32_t width, int32_t relu, void* hip_stream);
/* Scratch (float32 count) that tomo_nn_conv3x3_wgrad needs for npx = batch*height*width. */
tomo_status tomo_nn_wgrad_scratch(int32_t cin, int32_t cout, int32_t npx, size_t* floats);
/* dw [cout][3][3][cin] = sum over pixels of dz[p][co] x[p + tap][ci] (zero padding) and
 * db [cout] = sum over pixels of dz[p][co], float32, deterministic (fixed-order split sums).
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, HIP. */
tomo_status tomo_nn_conv3x3_wgrad(const uint16_t* dz, int32_t ldz, const uint16_t* x, int32_t ldx,
                                  float* dw, float* db, int32_t cin, int32_t cout, int32_t batch,
                                  int32_t height, int32_t width, float* scratch,
                                  size_t scratch_floats, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): tomo_nn_conv3x3_wgrad with the split partial sums in
 * a static device array of TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS floats (36 MiB) that the library
 * holds on every GPU it runs on until the process ends, instead of caller scratch.  Same
 * arguments, kernels and bit-identical results otherwise.  The caller still passes dz, x, dw
 * and db; hip_stream must belong to the current device.  The first call on a device looks up
 * the array's address on that device.  Calls that overlap on one GPU (other streams, other threads) share the
 * array and race; serialise them.  Errors: INVALID_ARG, WORKSPACE_TOO_SMALL (the shape needs more
 * split sums than the array holds; tomo_nn_wgrad_scratch gives the count), HIP. */
#define TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS 9437184
tomo_status tomo_nn_conv3x3_wgrad_noalloc(const uint16_t* dz, int32_t ldz, const uint16_t* x,
                                          int32_t ldx, float* dw, float* db, int32_t cin,
                                          int32_t cout, int32_t batch, int32_t height,
                                          int32_t width, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_NN_H */
