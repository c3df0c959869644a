// Host-side bounds check of the per-object crop loads (test infrastructure).
// Reads boxes from stdin -- a header "w h pitch count", then count lines
// "x0 y0 x1 y1" -- and walks every load the per-object kernels issue for each
// box: the three plane strides in use (R + 1 for the register classes when
// the crop fits them, cw | 1 otherwise), every thread count in use, every
// batch and every load of a batch, through the kernels' own address function
// (crop_addr.h), the loads of the erase pass, and the dense loads of the
// register classes (crops of at most 32 x 32 and 64 x 64, 64 and 128 threads).  Each offset must address a
// pixel of the crop, and so lie in [0, (h - 1) * pitch + w).  The dense row
// of every pixel of every crop of at most 64 x 64 is checked against integer
// division first.  Prints "ok <loads>" or the first failure.
#include <cstdio>

#include "crop_addr.h"

using namespace rtseg;

// the dense row of every crop pixel of every crop of at most 64 x 64
static bool dense_rows_exact() {
    for (int cw = 1; cw <= 64; ++cw) {
        const float inv = 1.0f / (float)cw;
        for (int k = 0; k < cw * 64; ++k)
            if (crop_dense_row(k, inv) != k / cw) {
                printf("FAIL dense row k %d cw %d: %d\n", k, cw, crop_dense_row(k, inv));
                return false;
            }
    }
    return true;
}

int main() {
    if (!dense_rows_exact()) return 1;
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
        // erase pass: lane = column, rows in batches of eight, clamped
        for (int c = 0; c < base.cw; ++c)
            for (int r0 = 0; r0 < base.ch; r0 += 8)
                for (int k = 0; k < 8; ++k) {
                    const long long o = crop_erase_offset(base, c, r0 + k, pitch);
                    const long long y = o / pitch, x = o % pitch;
                    ++loads;
                    if (o < 0 || o >= end || x < base.cx0 || x >= base.cx0 + base.cw || y < base.cy0 ||
                        y >= base.cy0 + base.ch) {
                        printf("FAIL erase box %d (%d %d %d %d) c %d r %d: offset %lld\n", b, x0, y0, x1, y1, c, r0 + k, o);
                        return 1;
                    }
                }
        // dense loads of the register classes (64 threads for 32 x 32, 128 for 64 x 64)
        for (int rc = 0; rc < 2; ++rc) {
            const int R = rc ? 64 : 32, nt = rc ? 128 : 64;
            if (base.cw > R || base.ch > R) continue;
            const float inv = 1.0f / (float)base.cw;
            const int npx = base.cw * base.ch;
            for (int k0 = 0; k0 < npx; k0 += LOADS_IN_FLIGHT * nt)
                for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
                    for (int lane = 0; lane < nt; ++lane) {
                        const long long o = crop_load_offset_dense(base, k0 + k * nt + lane, inv, pitch);
                        const long long y = o / pitch, x = o % pitch;
                        ++loads;
                        if (o < 0 || o >= end || x < base.cx0 || x >= base.cx0 + base.cw || y < base.cy0 ||
                            y >= base.cy0 + base.ch) {
                            printf("FAIL dense box %d (%d %d %d %d) threads %d k0 %d k %d lane %d: offset %lld\n", b,
                                   x0, y0, x1, y1, nt, k0, k, lane, o);
                            return 1;
                        }
                    }
        }
    }
    printf("ok %lld\n", loads);
    return 0;
}
