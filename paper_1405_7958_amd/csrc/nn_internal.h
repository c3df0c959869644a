// Internal declarations of the U-Net surrogate: layer kernels (k_nn.hip) and
// the network object (unet.cpp).
//
// Activations are NHWC bfloat16 (channel counts multiples of 8; the RGB input
// is padded to 8 channels), gradients of activations NHWC float32.  Weights
// are kept in float32 master copies in the layouts below, from which the
// bfloat16 operand copies of the matrix-core kernels are packed:
//   conv3 weights  [co][9][ci]   (tap = 3*ky + kx; ci padded to 8)
//   up2 weights    [ci][4][co]   (ab = 2*a + b: output pixel (2i+a, 2j+b))
//   head weights   [2][16]
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rtseg {

typedef uint16_t bf16_t;   // bfloat16 storage

// ---- matrix-core layers -----------------------------------------------------
// y = conv3(x0 ++ x1) (concatenated along channels) + bias, optional ReLU.
// Output bfloat16 (y, nullable) and/or float32 (yf, nullable).
int nn_conv3_fwd(const bf16_t *x0, int c0, const bf16_t *x1, int c1, int n, int h, int w, const bf16_t *wk,
                 const float *bias, int co, int relu, bf16_t *y, float *yf, hipStream_t s);
// dx = conv3 transpose of g (NHWC, co channels) with wt = [ci][9][co]; the
// ci output columns are split: [0, c0) -> dx0, [c0, ci) -> dx1 (nullable when
// c0 == ci).  float32 outputs, overwritten.
int nn_conv3_dgrad(const bf16_t *g, int co, int n, int h, int w, const bf16_t *wt, int ci, int c0, float *dx0,
                   float *dx1, hipStream_t s);
// dw[co][9][ci] += sum over pixels g[p][co] * (x0 ++ x1)[p + tap offset][ci]
int nn_conv3_wgrad(const bf16_t *x0, int c0, const bf16_t *x1, int c1, const bf16_t *g, int co, int n, int h, int w,
                   float *dw, hipStream_t s);
// y (n, 2h, 2w, co) = up2(x (n, h, w, ci)) + bias with uf = [4][co][ci]
int nn_up2_fwd(const bf16_t *x, int ci, int n, int h, int w, const bf16_t *uf, const float *bias, int co, bf16_t *y,
               float *yf, hipStream_t s);
// dx (n, h, w, ci) = up2 transpose of g (n, 2h, 2w, co) with ut = [ci][4][co]
int nn_up2_dgrad(const bf16_t *g, int co, int n, int h, int w, const bf16_t *ut, int ci, float *dx, hipStream_t s);
// dw[ci][4][co] += sum over input pixels x[p][ci] * g[(2i+a, 2j+b)][co]
int nn_up2_wgrad(const bf16_t *x, int ci, const bf16_t *g, int co, int n, int h, int w, float *dw, hipStream_t s);

// ---- element-wise layers ------------------------------------------------------
// db[c] += sum over pixels of g[p][c]
int nn_colsum(const bf16_t *g, int c, int64_t pixels, float *db, hipStream_t s);
// g = bf16(dy * (y > 0)) (y nullable: plain conversion)
int nn_relu_bwd(const float *dy, const bf16_t *y, int64_t count, bf16_t *g, hipStream_t s);
// 2x2 max pooling; idx = position of the maximum in the window (first on ties)
int nn_pool2_fwd(const bf16_t *x, int c, int n, int h, int w, bf16_t *y, uint8_t *idx, hipStream_t s);
// dx (n, h, w, c) += unpool(dy (n, h/2, w/2, c))
int nn_pool2_bwd(const float *dy, const uint8_t *idx, int c, int n, int h, int w, float *dx, hipStream_t s);
// RGB uint8 windows -> bfloat16 input (value / 255 - 0.5, channels 3..7 zero).
// Window k of the batch starts at (ox[k], oy[k]) of an RGB image (rgb, pitch
// in bytes, iw x ih); pixels outside the image read as 0 (before scaling).
int nn_prep_input(const uint8_t *rgb, int64_t pitch, int iw, int ih, const int32_t *ox, const int32_t *oy, int n,
                  int h, int w, bf16_t *x, hipStream_t s);
// 1x1 head + loss.  z = W x + b per pixel (2 maps).  With targets (training):
// loss_acc += sum of BCE terms / count (fg) + w_seed * ... (seed), dx = d/dx,
// dw, db accumulated.  Without targets (inference): probabilities sigmoid(z)
// are written to the window interiors of the output maps.
struct HeadArgs {
    const bf16_t *x;                    // (n, h, w, 16)
    int n, h, w;
    const float *wh, *bh;               // [2][16], [2]
    const uint8_t *t_fg, *t_seed;       // (n, h, w) targets, nullable
    float w_seed;
    float *loss;                        // accumulated
    float *dx;                          // (n, h, w, 16)
    float *dw, *db;                     // accumulated
    // inference output
    float *p_fg, *p_seed;               // output maps, pitch `pitch` floats
    int64_t pitch;
    const int32_t *ox, *oy;             // window origins
    const int32_t *keep;                // per window: x0, x1, y0, y1 kept (window coordinates)
    int out_w, out_h;
};
int nn_head(const HeadArgs &a, hipStream_t s);
// Adam over a flat parameter vector (bias-corrected, step t >= 1); zeroes g.
int nn_adam(float *p, float *g, float *m, float *v, int64_t count, float lr, float b1, float b2, float eps, int t,
            hipStream_t s);
// bfloat16 operand copies of a conv3 weight [co][9][ci]: wf = same layout,
// wt = [ci][9][co]
int nn_pack_conv3(const float *w, int co, int ci, bf16_t *wf, bf16_t *wt, hipStream_t s);
// bfloat16 operand copies of an up2 weight [ci][4][co]: uf = [4][co][ci], ut = same layout
int nn_pack_up2(const float *w, int ci, int co, bf16_t *uf, bf16_t *ut, hipStream_t s);
int nn_fill_f32(float *p, float v, int64_t n, hipStream_t s);

}  // namespace rtseg
