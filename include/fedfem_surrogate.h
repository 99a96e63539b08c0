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
 * Create a network for grid size G (a multiple of 4, from 4 to 256) and up
 * to batch_max samples per call (1 to 4096, with batch_max G^3 below 2^31),
 * with He-initialised weights from a seeded counter-based generator.
 * Allocates all activation, gradient and optimiser buffers on the current
 * device.  FEDFEM_E_INVALID for sizes outside these bounds.
 */
int fedsur_create(int32_t grid, int32_t batch_max, uint64_t seed,
                  fedsur_net **out);
int fedsur_destroy(fedsur_net *n);

/*
 * Stream for the network's kernels.  A new network uses a stream of its own
 * that is ordered with the legacy default stream (not a non-blocking one),
 * so inputs written there are complete before the network reads them.
 * stream = NULL selects the legacy default stream itself.  Every network
 * entry point synchronises this stream before it returns.
 */
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
 * Forward pass, weighted mean-squared error L = sum m (y - t)^2 / sum m over
 * the batch (m: a 0/1 mask or non-negative weights), and the backward pass
 * into the gradient vector.  target and mask are FP32 [B][G^3] device
 * arrays; loss (host, may be NULL) receives L.
 */
int fedsur_loss_backward(fedsur_net *n, int32_t batch, const void *x,
                         const float *target, const float *mask, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the held gradients. */
int fedsur_adam_step(fedsur_net *n, float lr);

/* Post-ReLU output of convolution `layer` (0..9) as FP32, host [B][g^3][C]. */
int fedsur_read_activation(fedsur_net *n, int32_t layer, float *host);

/*
 * One surrogate sample: the source, the material parameters and the domain
 * of one scenario (SI units).  The domain is the ellipsoid with semi-axes
 * (ax, ay, az) centred on the voxel frame; hmesh is the spacing of the
 * FED-FEM mesh whose results the network learns.
 */
typedef struct fedsur_sample {
    double cx, cy, cz; /* source centre [m] */
    double sigma;      /* source width [m] (> 0) */
    double q0;         /* source peak power density [W/m^3] */
    double k0;         /* conductivity at the reference temperature [W/(m K)] (> 0) */
    double omega_b;    /* perfusion rate [1/s] */
    double ax, ay, az; /* ellipsoid semi-axes [m] */
    double hmesh;      /* FED-FEM mesh spacing [m] */
    double reserved;   /* unused, keeps the record at 96 bytes */
} fedsur_sample;

/* Constants shared by a batch: density, specific heat at the reference
 * temperature, blood density times blood specific heat, heating time. */
typedef struct fedsur_phys {
    double rho0, c0, rhob_cb, t_heat;
} fedsur_phys;

/*
 * Network input, prior and scale for `batch` samples on a G^3 grid of cubic
 * voxels; frame = (x0, y0, z0, h) is the grid's lower corner and voxel edge
 * [m] (host array).  samples: device array [batch]; phys: host.
 *
 * The prior is the closed-form temperature rise of the sample's Gaussian
 * source Q0 exp(-|x - c|^2 / (2 sigma^2)), switched on at t = 0 and held
 * for t_heat, in an infinite medium of constant properties (k0, rho0 c0)
 * with perfusion omega_b rho_b c_b, i.e. the Pennes equation (Eq. 1)
 * without boundaries or temperature dependence.  It is evaluated at every
 * voxel centre in FP64 (an 8-point Gauss-Legendre rule on 8 geometric
 * pieces of [0, t_heat]) and stored as FP32 in prior [batch][G^3] (device,
 * may be NULL when not needed); scale [batch] (device) receives its value
 * at the source centre, P.  The network learns (dT - prior) / P.
 *
 * x (BF16 device [batch][G^3][8]) channels: 0 the voxel average of the
 * source shape exp(-|x - c|^2 / (2 sigma^2)), 1 (k0 - 0.525) / 0.075,
 * 2 (omega_b - 0.011) / 0.009, 3 the ellipsoid mask (voxel centre inside),
 * 4 prior / P, 5 prior / 100 K, 6 hmesh / 2 mm - 1, 7 sigma / 4 mm - 1;
 * channels 1-3 and 5-7 are zero outside the mask.
 *
 * Asynchronous on `stream` (NULL: the default stream).  Sample values live
 * in device memory and are not checked: sigma <= 0 or k0 <= 0 give
 * non-finite outputs, never an out-of-range access.
 */
int fedsur_rasterize(int32_t grid, const double *frame, int32_t batch,
                     const fedsur_sample *samples, const fedsur_phys *phys,
                     void *x, float *prior, float *scale, void *stream);

/*
 * Training target from FED-FEM temperatures resampled onto the grid
 * (fedfem_resample): target = (T - T_a - prior) / P where mask is set and 0
 * elsewhere, and the loss weight 1 + focus max(prior / P, 0) where mask is
 * set and 0 elsewhere (focus >= 0; 0 gives the plain mask), which leans
 * the masked mean-squared error (fedsur_loss_backward) towards the heated
 * region where the largest errors lie.  All arrays [batch][G^3] on the
 * device; asynchronous on `stream`.
 */
int fedsur_target(int32_t grid, int32_t batch, const float *prior,
                  const float *scale, const float *T, const uint8_t *mask,
                  float T_a, float focus, float *target, float *weight,
                  void *stream);

/*
 * Predicted temperature from the network's output y (fedsur_forward), in
 * place: y <- T_a + prior + P y (device arrays [batch][G^3]; asynchronous).
 */
int fedsur_decode(int32_t grid, int32_t batch, const float *prior,
                  const float *scale, float T_a, float *y, void *stream);

/*
 * err[b] (device, FP32) = max over voxels with mask set of |Tp[b] - T[b]|:
 * a predicted temperature field against FED-FEM's (fedfem_resample) for
 * each sample, 0 for a sample with an empty mask, NaN if any compared value
 * is NaN.  Asynchronous on `stream`; batch <= 65535.
 */
int fedsur_max_error(int32_t grid, int32_t batch, const float *Tp,
                     const float *T, const uint8_t *mask, float *err,
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
