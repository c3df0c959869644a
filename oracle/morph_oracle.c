/*
 * morph_oracle.c -- plain CPU oracle of the pre-processing operations the
 * paper lists beside the segmentation (Sec. 5.1: Morphological Open, RBC
 * detection; the ReconToNuclei marker).  TEST INFRASTRUCTURE ONLY (see
 * rt_oracle.h).  Every function is its definition written out with plain
 * loops; definitions and readings are in rt_oracle.h.
 */
#include <stdlib.h>
#include <string.h>

#include "rt_oracle.h"

/* flat disk: offsets (dx, dy) with dx^2 + dy^2 <= r^2 */
static int in_disk(int dx, int dy, int r) { return dx * dx + dy * dy <= r * r; }

void or_erode(const uint8_t *in, int w, int h, int radius, uint8_t *out) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int m = 255;
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    const int xx = x + dx, yy = y + dy;
                    if (!in_disk(dx, dy, radius) || xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
                    const int v = in[(int64_t)yy * w + xx];
                    if (v < m) m = v;
                }
            out[(int64_t)y * w + x] = (uint8_t)m;
        }
}

void or_dilate(const uint8_t *in, int w, int h, int radius, uint8_t *out) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int m = 0;
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    const int xx = x + dx, yy = y + dy;
                    if (!in_disk(dx, dy, radius) || xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
                    const int v = in[(int64_t)yy * w + xx];
                    if (v > m) m = v;
                }
            out[(int64_t)y * w + x] = (uint8_t)m;
        }
}

void or_open(const uint8_t *in, int w, int h, int radius, uint8_t *out) {
    uint8_t *t = (uint8_t *)malloc((size_t)w * h);
    or_erode(in, w, h, radius, t);
    or_dilate(t, w, h, radius, out);
    free(t);
}

void or_recon_to_nuclei(const uint8_t *hq, int w, int h, int marker_mode, int radius, int t_fg, uint8_t *recon_out,
                        uint8_t *f0_out) {
    const int64_t N = (int64_t)w * h;
    int32_t *mk = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *ms = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *r = (int32_t *)malloc(sizeof(int32_t) * N);
    if (marker_mode == OR_MARKER_OPEN) {
        uint8_t *e = (uint8_t *)malloc((size_t)N);
        or_erode(hq, w, h, radius, e);
        for (int64_t i = 0; i < N; ++i) mk[i] = e[i];
        free(e);
    } else {
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                const int64_t i = (int64_t)y * w + x;
                mk[i] = (x == 0 || y == 0 || x == w - 1 || y == h - 1) ? hq[i] : 0;
            }
    }
    for (int64_t i = 0; i < N; ++i) ms[i] = hq[i];
    or_recon(mk, ms, NULL, w, h, 8, r);
    for (int64_t i = 0; i < N; ++i) {
        if (recon_out) recon_out[i] = (uint8_t)r[i];
        f0_out[i] = (hq[i] - r[i] >= t_fg) ? 1 : 0;
    }
    free(mk);
    free(ms);
    free(r);
}

void or_rbc_detect(const uint8_t *rgb, int w, int h, int t_strong, int t_weak, uint8_t *mask_out) {
    const int64_t N = (int64_t)w * h;
    int32_t *mk = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *ms = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *r = (int32_t *)malloc(sizeof(int32_t) * N);
    for (int64_t i = 0; i < N; ++i) {
        const int red = 2 * rgb[3 * i] - rgb[3 * i + 1] - rgb[3 * i + 2];
        ms[i] = red >= t_weak ? 1 : 0;
        mk[i] = (red >= t_strong && ms[i]) ? 1 : 0;
    }
    /* the weak regions that hold a strong pixel: binary reconstruction */
    or_recon(mk, ms, NULL, w, h, 8, r);
    for (int64_t i = 0; i < N; ++i) mask_out[i] = (uint8_t)r[i];
    free(mk);
    free(ms);
    free(r);
}
