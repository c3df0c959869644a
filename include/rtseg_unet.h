/*
 * rtseg_unet.h -- C ABI of the learned surrogate of librtseg.so: a small
 * U-Net that predicts the foreground and seed maps of the segmentation stage
 * (Sec. 5.1 of Teodoro et al., "Region Templates"), trained on masks that the
 * plain pipeline produces, and a segmentation entry point that uses it with
 * the plain pipeline as fallback.  The paper has no learned component: the
 * surrogate replaces the reconstruction (ReconToNuclei) and the watershed
 * seeding, and every other step is the plain pipeline's own kernel.
 *
 * Network: 3x3 convolutions (zero padding) with ReLU, two per level, 16, 32,
 * 64 and 128 channels; 2x2 max pooling between encoder levels (ties to the
 * first element in row-major window order); decoder levels with a 2x2
 * stride-2 transposed convolution, concatenation [up-convolution output,
 * encoder skip] and two 3x3 convolutions with ReLU; a 1x1 head to two logit
 * maps (foreground, seeds).  Input: value / 255 - 0.5 per RGB channel.
 * Weights and activations bfloat16 (round to nearest even), products
 * accumulated in float32; float32 master weights updated by Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).  Loss: mean binary
 * cross-entropy with logits of the foreground map plus w_seed times that of
 * the seed map.
 *
 * Conventions are those of rtseg.h: device pointers, asynchronous on
 * `stream` unless noted, 0 = RT_OK, negative = error with rt_last_error().
 */
#ifndef RTSEG_UNET_H
#define RTSEG_UNET_H
#include <stdint.h>

#include "rtseg.h"
#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_unet rt_unet;

/*
 * Parameter vector: float32, in this order for every layer e1a e1b e2a e2b
 * e3a e3b e4a e4b u3 d3a d3b u2 d2a d2b u1 d1a d1b head: weights then bias.
 *   3x3 convolution weights  [co][9][ci]   tap = 3*ky + kx, (ky, kx) = row and
 *                                          column offset + 1; e1a has ci = 8,
 *                                          input channels 3..7 are zero
 *   up-convolution weights   [ci][4][co]   index 2*a + b writes output pixel
 *                                          (2i + a, 2j + b) from input (i, j)
 *   head weights             [2][16]       row 0 foreground, row 1 seeds
 */
int64_t rt_unet_param_count(void);

/* Creates a network on the context's device with He-normal weights drawn by
 * a counter-based generator (splitmix64 + Box-Muller) from `seed`. */
int rt_unet_create(rt_ctx *ctx, uint64_t seed, rt_unet **out);
int rt_unet_destroy(rt_unet *net);
/* Host copies of the parameters / of the accumulated gradients (count =
 * rt_unet_param_count()).  set_params also clears the Adam moments and the
 * step counter.  These synchronise the device. */
int rt_unet_get_params(rt_unet *net, float *host, int64_t count);
int rt_unet_set_params(rt_unet *net, const float *host, int64_t count);
int rt_unet_get_grads(rt_unet *net, float *host, int64_t count);

/*
 * Loss and gradient of a batch: rgb is b images of h x w x 3 bytes (dense),
 * fg_tgt and seed_tgt b x h x w bytes (0/1); h and w multiples of 8.  Writes
 * the loss to loss_dev (device float) and ADDS the gradients to the
 * accumulator (rt_unet_get_grads).  Synchronises `stream` at the end.
 * rt_unet_train_step does the same, then one Adam step with learning rate
 * lr, which also clears the accumulator.
 */
int rt_unet_grad_step(rt_unet *net, const uint8_t *rgb, const uint8_t *fg_tgt, const uint8_t *seed_tgt, int32_t b,
                      int32_t h, int32_t w, float w_seed, float *loss_dev, void *stream);
int rt_unet_train_step(rt_unet *net, const uint8_t *rgb, const uint8_t *fg_tgt, const uint8_t *seed_tgt, int32_t b,
                       int32_t h, int32_t w, float lr, float w_seed, float *loss_dev, void *stream);
/*
 * One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected with the step number t, which this call increments) on the FP32
 * master weights from the accumulated gradient, which it then clears, and a
 * repack of the bf16 operand copies: gradient accumulation over several
 * rt_unet_grad_step calls followed by one update.  Asynchronous on `stream`.
 * rt_unet_get_step returns t (0 after create or set_params).
 */
int rt_unet_adam_step(rt_unet *net, float lr, void *stream);
int rt_unet_get_step(rt_unet *net, int64_t *step);

/*
 * Tile inference: 512 x 512 windows at stride 480 (the last window flush with
 * the tile edge; along an axis shorter than 512 the window is the axis length
 * rounded up to a multiple of 8, the extra pixels reading as zero input);
 * each output pixel comes from the window whose kept part holds it, the
 * overlap of two windows being split at its middle.  fg_prob and seed_prob
 * are float maps (sigmoid of the logits) with pitch prob_pitch (elements).
 * The windows run in groups of 16 back to back; the window origins of the
 * whole tile are uploaded once, so the call waits on the host only for the
 * previous call's origin upload (if still pending).
 */
int rt_unet_forward(rt_unet *net, const uint8_t *rgb, int64_t rgb_pitch, int32_t w, int32_t h, float *fg_prob,
                    float *seed_prob, int64_t prob_pitch, void *stream);

/* Parameter file: 8 magic bytes "RTUNET01", int64 count, count float32. */
int rt_unet_save(rt_unet *net, const char *path);
int rt_unet_load(rt_unet *net, const char *path);
/* Training checkpoint, for resuming: 8 magic bytes "RTUNETC1", int64 count,
 * int64 step t, then count float32 each of the master weights, the gradient
 * accumulator, Adam's first and second moments.  Loading restores all of it
 * (and repacks the bf16 operand copies).  Both synchronise the device.
 * Errors: RT_EINVAL for a file that is not a checkpoint of this network. */
int rt_unet_save_checkpoint(rt_unet *net, const char *path);
int rt_unet_load_checkpoint(rt_unet *net, const char *path);

/*
 * Segmentation stage with the surrogate: fg = [p_fg >= 0.5], seeds =
 * [p_seed >= 0.5]; F = FillHoles(fg, 4); BWLabel; components with area >=
 * min_area; watershed of them from the network's seeds (rt_watershed with
 * external seeds); cut, relabel and keep [min_area, max_area] -- the last
 * steps of rt_segment_tile.  Confidence = 1 - max(u_fg, u_seed) with
 * u_m = #(0.25 <= p_m < 0.75) / #(p_m >= 0.25), the share of undecided
 * pixels among the likely-positive ones of each map; a tile with
 * confidence < tau is segmented by the plain
 * pipeline instead (*used_fallback = 1).  used_fallback and confidence are
 * host pointers (nullable); the call synchronises `stream` to read the
 * confidence.  Outputs as rt_segment_tile.
 */
int rt_segment_tile_surrogate(rt_ctx *ctx, rt_unet *net, const uint8_t *rgb, int64_t rgb_pitch, int32_t w,
                              int32_t h, const rt_seg_params *params, float tau, uint8_t *mask_out,
                              int32_t *labels_out, int64_t out_pitch, int32_t *n_objects_dev,
                              int32_t *used_fallback, float *confidence, void *stream);

/*
 * Single layers, for parity tests against the CPU oracle.  Activations NHWC
 * bfloat16 (uint16 storage), channel counts multiples of 8 (outputs of the
 * matrix-core layers multiples of 16, at most 128); results float32.
 *   conv3_fwd    y = conv3(x0 ++ x1) + bias, ReLU if relu; wf = [co][9][c0+c1]
 *   conv3_dgrad  dx = transpose conv of g (co channels) with wt = [ci][9][co];
 *                columns [0, c0) -> dx0, [c0, ci) -> dx1
 *   conv3_wgrad  dw[co][9][c0+c1] += ..., db[co] += sum of g (db nullable)
 *   up2_fwd      y (n, 2h, 2w, co) with uf = [4][co][ci]
 *   up2_bwd      dx (n, h, w, ci) = transpose with ut = [ci][4][co]; dw[ci][4][co]
 *                += ...; db += column sums of g (n, 2h, 2w, co); outputs nullable
 *   pool2        forward (x, y, idx) or backward (dy, idx, dx += unpool(dy))
 *   head_loss    1x1 head, loss (added to *loss), dx (n, h, w, 16) written,
 *                dw [2][16] and db [2] accumulated
 *   pack         bfloat16 operand copies: kind 0 conv3 [co][9][ci] -> fwd
 *                [co][9][ci] and tr [ci][9][co]; kind 1 up2 [ci][4][co] -> fwd
 *                [4][co][ci] and tr [ci][4][co]
 *   prep_input   RGB bytes (pitch in bytes) -> (h, w, 8) network input
 */
int rt_nn_conv3_fwd(rt_ctx *ctx, const uint16_t *x0, int32_t c0, const uint16_t *x1, int32_t c1, int32_t n,
                    int32_t h, int32_t w, const uint16_t *wf, const float *bias, int32_t co, int32_t relu, float *y_f32,
                    uint16_t *y_bf16, void *stream);
int rt_nn_conv3_dgrad(rt_ctx *ctx, const uint16_t *g, int32_t co, int32_t n, int32_t h, int32_t w, const uint16_t *wt,
                      int32_t ci, int32_t c0, float *dx0, float *dx1, void *stream);
int rt_nn_conv3_wgrad(rt_ctx *ctx, const uint16_t *x0, int32_t c0, const uint16_t *x1, int32_t c1, const uint16_t *g,
                      int32_t co, int32_t n, int32_t h, int32_t w, float *dw, float *db, void *stream);
int rt_nn_up2_fwd(rt_ctx *ctx, const uint16_t *x, int32_t ci, int32_t n, int32_t h, int32_t w, const uint16_t *uf,
                  const float *bias, int32_t co, float *y_f32, uint16_t *y_bf16, void *stream);
int rt_nn_up2_bwd(rt_ctx *ctx, const uint16_t *x, int32_t ci, const uint16_t *g, int32_t co, int32_t n, int32_t h,
                  int32_t w, const uint16_t *ut, float *dx, float *dw, float *db, void *stream);
int rt_nn_pool2(rt_ctx *ctx, const uint16_t *x, int32_t c, int32_t n, int32_t h, int32_t w, uint16_t *y, uint8_t *idx,
                const float *dy, float *dx, void *stream);
int rt_nn_head_loss(rt_ctx *ctx, const uint16_t *x, int32_t n, int32_t h, int32_t w, const float *wh, const float *bh,
                    const uint8_t *t_fg, const uint8_t *t_seed, float w_seed, float *loss, float *dx, float *dw,
                    float *db, void *stream);
int rt_nn_pack(rt_ctx *ctx, int32_t kind, const float *w, int32_t ci, int32_t co, uint16_t *fwd, uint16_t *tr,
               void *stream);
int rt_nn_prep_input(rt_ctx *ctx, const uint8_t *rgb, int64_t pitch, int32_t w, int32_t h, uint16_t *x, void *stream);

#ifdef __cplusplus
}
#endif
#endif
