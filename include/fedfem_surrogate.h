/*
 * fedfem_surrogate.h -- C ABI of the learned surrogate for FED-FEM runs.
 *
 * A 3-level 3-D convolutional encoder-decoder on a G^3 voxel grid maps a
 * rasterised source-power field, the conductivity and perfusion parameters
 * and the domain's occupancy mask to the temperature rise after a fixed
 * heating time.  Layers: two 3x3x3 convolutions with ReLU per level
 * (32, 64, 128 channels), 2x2x2 average pooling down, nearest-neighbour 2x
 * upsampling up, skip connections by channel concatenation, a 1x1x1 output
 * head.  Weights are kept in FP32 (Adam master copy) and used as BF16 by
 * the MFMA kernels, which accumulate in FP32.  FED-FEM (fedfem.h) produces
 * the training targets, is the fallback and judges the surrogate's error.
 *
 * Tensors are channels-last ("NDHWC"): [B][G][G][G][C], voxel (z, y, x).
 * Device pointers are plain HIP device memory; BF16 values are passed as
 * 16-bit words (void *).  Return codes are those of fedfem.h.
 */
#ifndef FEDFEM_SURROGATE_H
#define FEDFEM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "fedfem.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FEDSUR_IN_CHANNELS 8 /* source, k0, perfusion, mask, 4 zero pads */
#define FEDSUR_LAYERS 10     /* 3x3x3 convolutions, then the 1x1x1 head  */

typedef struct fedsur_net fedsur_net;

/*
 * Create a network for grid size G (a multiple of 4, at least 4) and up to
 * batch_max samples per call, with He-initialised weights from a seeded
 * counter-based generator.  Allocates all activation, gradient and
 * optimiser buffers on the current device.
 */
int fedsur_create(int32_t grid, int32_t batch_max, uint64_t seed,
                  fedsur_net **out);
int fedsur_destroy(fedsur_net *n);
int fedsur_set_stream(fedsur_net *n, void *stream);

/*
 * Parameters as one FP32 vector: for each convolution in order (e1a, e1b,
 * e2a, e2b, e3a, e3b, d2a, d2b, d1a, d1b) its weights [Cout][3][3][3][Cin]
 * then its biases [Cout], then the head's weights [32] and bias [1].
 */
int fedsur_param_count(const fedsur_net *n, int64_t *count);
int fedsur_get_params(fedsur_net *n, float *host);
int fedsur_set_params(fedsur_net *n, const float *host); /* resets Adam */
int fedsur_get_grads(fedsur_net *n, float *host);

/* y [B][G^3] (FP32, device) from x [B][G^3][8] (BF16, device). */
int fedsur_forward(fedsur_net *n, int32_t batch, const void *x, float *y);

/*
 * Forward pass, masked mean-squared error L = sum m (y - t)^2 / sum m over
 * the batch, and the backward pass into the gradient vector.  target and
 * mask are FP32 [B][G^3] device arrays; loss (host, may be NULL) receives L.
 */
int fedsur_loss_backward(fedsur_net *n, int32_t batch, const void *x,
                         const float *target, const float *mask, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the held gradients. */
int fedsur_adam_step(fedsur_net *n, float lr);

/* Post-ReLU output of convolution `layer` (0..9) as FP32, host [B][g^3][C]. */
int fedsur_read_activation(fedsur_net *n, int32_t layer, float *host);

/*
 * Network input on a G^3 grid of cubic voxels: frame = (x0, y0, z0, h), the
 * lower corner and voxel edge [m].  params per sample: (cx, cy, cz, sigma,
 * Q0, k0, omega_b).  Channel 0 is the voxel average of
 * Q0 exp(-|x - c|^2 / (2 sigma^2)) (a product of error-function differences)
 * times 1e-7, channel 1 (k0 - 0.525) / 0.075, channel 2
 * (omega_b - 0.011) / 0.009, channel 3 the occupancy mask (uint8 device
 * array [B][G^3]); channels 1-3 are zero outside the mask, 4-7 are zero.
 * x is BF16 [B][G^3][8] on the device.
 */
int fedsur_rasterize(int32_t grid, const double *frame, int32_t batch,
                     const double *params, const uint8_t *mask, void *x,
                     void *stream);

/*
 * Temperature of a precomputed handle at the voxel centres of a G^3 grid
 * (frame as above) by linear interpolation in the containing tetrahedron
 * (P1 shape functions); a voxel whose centre lies in several elements takes
 * the one with the smallest internal id.  T_out [G^3] (FP32, device) gets
 * T there and 0 outside the mesh; mask_out [G^3] (uint8, device) marks the
 * voxels inside.  Synchronises the handle's stream.
 */
int fedfem_resample(fedfem_handle *h, int32_t grid, const double *frame,
                    float *T_out, uint8_t *mask_out);

#ifdef __cplusplus
}
#endif

#endif /* FEDFEM_SURROGATE_H */
