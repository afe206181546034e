/*
 * libfibar learned stale fill: a small convolutional network that predicts
 * the brightness of stale pixels from a readout of the reconstruction, with
 * the blurred brightness the reconstruction already holds (the paper's one-time
 * 3x3 Gaussian fill of stale pixels, Method, "Spatial filtering") as the
 * per-tile fallback.  It is an addition to the paper's method: it reads a
 * readout and never writes into a reconstruction context, so the
 * reconstruction itself is unchanged.
 *
 * Network: four zero-padded 3x3 cross-correlation layers (no kernel flip),
 * channels 3 -> 16 -> 16 -> 16 -> 1, ReLU after the first three.  Input
 * channels per pixel: brightness L, stale mask (1 stale, 0 otherwise),
 * log(1 + age).  The prediction is L plus the last layer's output (a learned
 * correction of the brightness the reconstruction shows).  BF16 weights and
 * activations, FP32 MFMA accumulation, FP32 biases and FP32 master
 * parameters.  Training loss: the mean of (prediction - target)^2 over the
 * stale pixels of a batch; optimiser Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected).
 *
 * Parameters travel as one flat FP32 vector of FIBAR_FILL_PARAMS values,
 * layer by layer: w in [Cout][Cin][3][3] order, then b[Cout].
 *
 * Images: n images of H x W pixels, row-major, image after image; every
 * image pointer is a device pointer.  Calls are ordered on the stream given
 * at creation (NULL = null stream); the model's device buffers are owned by
 * the handle and grow to the largest n * H * W used.  Errors: the fibar_status
 * codes of fibar.h (FIBAR_E_INVALID_ARG for null pointers or zero sizes,
 * FIBAR_E_NOMEM, FIBAR_E_DEVICE).  Calls on one handle must not overlap.
 */
#ifndef FIBAR_FILL_H
#define FIBAR_FILL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FIBAR_FILL_PARAMS 5233

typedef struct fibar_fill fibar_fill;

/* A model with all parameters zero (set them with fibar_fill_set_params). */
int fibar_fill_create(void* stream, fibar_fill** out);

/* Host FP32 vectors of FIBAR_FILL_PARAMS values.  Setting the parameters
 * restarts Adam (zero moments, step 0); both calls synchronise the stream. */
int fibar_fill_set_params(fibar_fill* f, const float* params);
int fibar_fill_get_params(fibar_fill* f, float* params);

/* Prediction per pixel (L + the network's output) into pred (FP32, n * H * W). */
int fibar_fill_predict(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                       uint32_t n, uint32_t H, uint32_t W, float* pred);

/* Loss of a batch against `target` (FP32, n * H * W) over its stale pixels,
 * into *loss (host), and optionally the gradient of the loss with respect to
 * every parameter into `grad` (host, FIBAR_FILL_PARAMS, may be NULL).
 * Synchronises the stream.  A batch without stale pixels has loss 0 and a
 * zero gradient. */
int fibar_fill_loss_grad(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                         const float* target, uint32_t n, uint32_t H, uint32_t W, float* loss,
                         float* grad);

/* One Adam step on a batch with learning rate lr.  `loss` (host, may be
 * NULL) receives the batch loss before the step, which synchronises the
 * stream; with NULL the step is queued without waiting. */
int fibar_fill_train_step(fibar_fill* f, const float* L, const uint8_t* stale,
                          const float* log_age, const float* target, uint32_t n, uint32_t H,
                          uint32_t W, float lr, float* loss);

/* Filled image of one readout (H x W): L where the pixel is not stale; at
 * stale pixels the network's prediction in tiles of tile x tile pixels
 * (tile in 4..64; edge tiles cut by the image) where more than a fraction
 * theta (>= 0) of the tile's pixels are stale and every stale prediction is
 * finite; every other tile keeps L, the reconstruction's own one-time
 * Gaussian fill -- the per-tile fallback.  theta = 0 uses the network in
 * every tile with a stale pixel, theta >= 1 in none.  `fallback_tiles`
 * (host, may be NULL) receives the number of tiles with stale pixels that
 * kept L, which synchronises the stream.  The prediction buffer is owned by
 * the handle and grows to the largest H * W used. */
int fibar_fill_apply(fibar_fill* f, const float* L, const uint8_t* stale, const float* log_age,
                     uint32_t H, uint32_t W, uint32_t tile, float theta, float* out,
                     uint32_t* fallback_tiles);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as fibar_fill_apply, bit for bit, with no allocation at all.  The
 * prediction and the fallback counter live in a fixed device array of the
 * library, one per GPU (4 MiB + 256 bytes, looked up when a handle is created
 * on that GPU and held until the process ends), so H * W may be at most
 * 1048576 pixels (FIBAR_E_INVALID_ARG beyond).  Every call on a GPU uses that
 * GPU's array: calls that overlap on one GPU (on different streams, or from
 * different threads) race and must be serialised by the caller. */
int fibar_fill_apply_noalloc(fibar_fill* f, const float* L, const uint8_t* stale,
                             const float* log_age, uint32_t H, uint32_t W, uint32_t tile,
                             float theta, float* out, uint32_t* fallback_tiles);

void fibar_fill_destroy(fibar_fill* f);

#ifdef __cplusplus
}
#endif

#endif /* FIBAR_FILL_H */
