/*
 * ct_unet.h -- C ABI of the learned warm start of libctrlalm: a BF16 U-Net (4 levels, 32/64/128/256
 * channels, 3x3 convolutions on the gfx950 matrix cores with FP32 accumulation) that maps the
 * FBP-like image of a scan (ct_fbp, in units of mu_water) to a start image for the relaxed OS-LALM
 * solve (ct_rlalm_params.start = 3). Algorithm 1 of the paper takes any x0 in Omega and its experiments
 * start from FBP; the network refines that FBP image (an extension, not the paper's).
 *
 * Network (canonical order of the parameters; each layer: weight [c_out][c_in][k][k] float32, then
 * bias [c_out]):
 *   enc1a 1->32, enc1b 32->32, enc2a 32->64, enc2b 64->64, enc3a 64->128, enc3b 128->128,
 *   bottleneck 128->256, 256->256, dec3a 384->128 (256 upsampled + 128 skip), dec3b 128->128,
 *   dec2a 192->64 (128 + 64), dec2b 64->64, dec1a 96->32 (64 + 32), dec1b 32->32, out 1x1 32->1.
 *   Every 3x3 convolution is zero-padded and followed by ReLU; 2x2 average pooling between encoder
 *   levels; nearest 2x upsampling in the decoder; output = input + out-layer (residual). Images are in
 *   units of mu_water. Training loss: mean over a pixel mask of (1000 (output - target))^2 (HU^2),
 *   minimised by Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Conventions as in ct.h: device pointers owned by the caller, stream-ordered calls, ct_status
 * returns, ct_last_error() for the message. Image batches are float32 [n][h][w], h and w multiples
 * of 8. A handle is not safe for concurrent use from two streams.
 */
#ifndef CTRLALM_CT_UNET_H
#define CTRLALM_CT_UNET_H

#include <stddef.h>

#include "ct.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ct_unet ct_unet;

/* Number of float32 parameters (1,946,305). */
size_t ct_unet_num_params(void);

/*
 * Create a network on the current device for batches of up to max_n images of up to max_h x max_w
 * (multiples of 8), with parameters theta (HOST float32, ct_unet_num_params() values, canonical order).
 * Errors: CT_ERR_INVALID_ARG (NULL, sizes), CT_ERR_OOM, CT_ERR_HIP.
 */
ct_status ct_unet_create(const float *theta, int max_n, int max_h, int max_w, ct_unet **out);
void ct_unet_destroy(ct_unet *u);

/* Replace the parameters (HOST float32) and reset the optimiser state; read them back (synchronises). */
ct_status ct_unet_set_params(ct_unet *u, const float *theta);
ct_status ct_unet_get_params(const ct_unet *u, float *theta);

/* out = network(x): x and out are DEVICE float32 [n][h][w] (may not alias). */
ct_status ct_unet_forward(ct_unet *u, const float *x, float *out, int n, int h, int w, void *stream);

/*
 * Loss and gradient at the current parameters without an update. mask: DEVICE uint8 [h][w] (non-zero =
 * pixel counts), shared by the n images. loss (HOST, may be NULL): the loss in HU^2. grad (HOST, may be
 * NULL): ct_unet_num_params() float32 values in canonical order. Synchronises.
 */
ct_status ct_unet_gradient(ct_unet *u, const float *x, const float *target, const unsigned char *mask, int n, int h,
                           int w, double *loss, float *grad, void *stream);

/* One Adam step on the batch (forward, loss, backward, update); loss (HOST, may be NULL) is the loss
   before the update. Synchronises only when loss is requested. */
ct_status ct_unet_train_step(ct_unet *u, const float *x, const float *target, const unsigned char *mask, int n, int h,
                             int w, float lr, double *loss, void *stream);

/*
 * Network input of a scan: x_in = FBP-like image of y (ct_fbp) / mu_water, DEVICE float32 [ny][nx]; y in
 * the geometry's storage type. Flat detector only (CT_ERR_UNSUPPORTED otherwise). Uses the handle's
 * workspace (do not overlap with a solve on the same handle).
 */
ct_status ct_unet_input(ct_geom *g, const void *y, double mu_water, float *x_in, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CTRLALM_CT_UNET_H */
