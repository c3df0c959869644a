/*
 * stitch_oracle.c -- plain CPU oracle of cross-tile stitching with ghost
 * cells (Sec. 3.4: a partition of a data region is extended by ghost cells
 * taken from its neighbours, so that objects cut by a partition border are
 * seen whole).  TEST INFRASTRUCTURE ONLY (see rt_oracle.h); the definition
 * and readings are in rt_oracle.h.
 */
#include <limits.h>
#include <stdlib.h>
#include <string.h>

#include "rt_oracle.h"

int or_stitch_from_hq(const uint8_t *hq, int W, int H, int tile, int halo, int t_fg, int min_area, int max_area,
                      int h_seed, int32_t *labels_out, uint8_t *mask_out) {
    const int64_t N = (int64_t)W * H;
    for (int64_t i = 0; i < N; ++i) labels_out[i] = INT_MAX;
    int owned = 0;
    for (int ty = 0; ty * tile < H; ++ty)
        for (int tx = 0; tx * tile < W; ++tx) {
            /* the core [x0, x1) x [y0, y1) and the extended region, clipped */
            const int x0 = tx * tile, y0 = ty * tile;
            const int x1 = x0 + tile < W ? x0 + tile : W, y1 = y0 + tile < H ? y0 + tile : H;
            const int ex0 = x0 - halo > 0 ? x0 - halo : 0, ey0 = y0 - halo > 0 ? y0 - halo : 0;
            const int ex1 = x1 + halo < W ? x1 + halo : W, ey1 = y1 + halo < H ? y1 + halo : H;
            const int ew = ex1 - ex0, eh = ey1 - ey0;
            uint8_t *sub = (uint8_t *)malloc((size_t)ew * eh);
            uint8_t *m = (uint8_t *)malloc((size_t)ew * eh);
            int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)ew * eh);
            for (int y = 0; y < eh; ++y) memcpy(sub + (size_t)y * ew, hq + (int64_t)(ey0 + y) * W + ex0, (size_t)ew);
            or_segment_from_hq(sub, ew, eh, t_fg, min_area, max_area, h_seed, m, lab, NULL, NULL, NULL, NULL);
            for (int y = 0; y < eh; ++y)
                for (int x = 0; x < ew; ++x) {
                    const int32_t L = lab[(size_t)y * ew + x];
                    if (L <= 0) continue;
                    /* the nucleus' first pixel (its label's root) in slide coordinates */
                    const int rx = ex0 + (L - 1) % ew, ry = ey0 + (L - 1) / ew;
                    if (rx < x0 || rx >= x1 || ry < y0 || ry >= y1) continue;   /* owned by another tile */
                    const int32_t S = (int32_t)((int64_t)ry * W + rx + 1);
                    int32_t *o = labels_out + (int64_t)(ey0 + y) * W + ex0 + x;
                    if (S < *o) *o = S;
                    if (ex0 + x == rx && ey0 + y == ry) ++owned;
                }
            free(sub);
            free(m);
            free(lab);
        }
    for (int64_t i = 0; i < N; ++i) {
        if (labels_out[i] == INT_MAX) labels_out[i] = 0;
        if (mask_out) mask_out[i] = labels_out[i] ? 1 : 0;
    }
    return owned;
}
