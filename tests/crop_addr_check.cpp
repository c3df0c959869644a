// Host-side bounds check of the per-object crop loads (test infrastructure).
// Reads boxes from stdin -- a header "w h pitch count", then count lines
// "x0 y0 x1 y1" -- and walks every load the per-object kernels issue for each
// box: the three plane strides in use (R + 1 for the register classes when
// the crop fits them, cw | 1 otherwise), every thread count in use, every
// batch and every load of a batch, through the kernels' own address function
// (crop_addr.h).  Each offset must address a pixel of the crop, and so lie in
// [0, (h - 1) * pitch + w).  Prints "ok <loads>" or the first failure.
#include <cstdio>

#include "crop_addr.h"

using namespace rtseg;

int main() {
    int w, h, count;
    long long pitch;
    if (scanf("%d %d %lld %d", &w, &h, &pitch, &count) != 4) return 2;
    const long long end = (long long)(h - 1) * pitch + w;
    long long loads = 0;
    for (int b = 0; b < count; ++b) {
        int x0, y0, x1, y1;
        if (scanf("%d %d %d %d", &x0, &y0, &x1, &y1) != 4) return 2;
        const CropGeom base = crop_of_box(x0, y0, x1, y1, w, h);
        const int strides[3] = {33, 65, base.cw | 1};
        for (int si = 0; si < 3; ++si) {
            if (si == 0 && (base.cw > 32 || base.ch > 32)) continue;
            if (si == 1 && (base.cw > 64 || base.ch > 64)) continue;
            const CropGeom q = crop_with_stride(base, strides[si]);
            const int threads[3] = {64, 128, 256};
            for (int ti = 0; ti < 3; ++ti) {
                const int nt = threads[ti];
                for (int i0 = 0; i0 < q.n; i0 += LOADS_IN_FLIGHT * nt)
                    for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
                        for (int lane = 0; lane < nt; ++lane) {
                            const long long o = crop_load_offset(q, i0 + k * nt + lane, pitch);
                            const long long y = o / pitch, x = o % pitch;
                            ++loads;
                            if (o < 0 || o >= end || x < q.cx0 || x >= q.cx0 + q.cw || y < q.cy0 ||
                                y >= q.cy0 + q.ch) {
                                printf("FAIL box %d (%d %d %d %d) stride %d threads %d i0 %d k %d lane %d: "
                                       "offset %lld (x %lld, y %lld), crop x %d+%d y %d+%d\n",
                                       b, x0, y0, x1, y1, q.st, nt, i0, k, lane, o, x, y, q.cx0, q.cw, q.cy0, q.ch);
                                return 1;
                            }
                        }
            }
        }
    }
    printf("ok %lld\n", loads);
    return 0;
}
