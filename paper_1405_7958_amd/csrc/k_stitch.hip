// Cross-tile stitching with ghost cells (Sec. 3.4): every extended tile of a
// launch group has been segmented on its own; these kernels move the nuclei
// a core owns (those whose first pixel lies inside the core) into the slide
// label map with their slide labels, the smaller label winning where two
// cores' nuclei cover one pixel.
#include "rt_internal.h"

namespace rtseg {

namespace {

// one block row (blockIdx.y) per extended tile of the group
__global__ __launch_bounds__(256) void k_stitch(StitchGroup g) {
    const StitchTile t = g.t[blockIdx.y];
    const int64_t n = (int64_t)t.ew * t.eh;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ey = (int)(i / t.ew), ex = (int)(i - (int64_t)ey * t.ew);
        const int sx = t.ex0 + ex, sy = t.ey0 + ey;
        const bool core = sx >= t.x0 && sx < t.x1 && sy >= t.y0 && sy < t.y1;
        if (g.hq_out && core) g.hq_out[(int64_t)sy * g.out_pitch + sx] = t.hq[i];
        const int32_t L = t.labels[i];
        if (L <= 0) continue;
        const int rx = t.ex0 + (L - 1) % t.ew, ry = t.ey0 + (L - 1) / t.ew;
        if (rx < t.x0 || rx >= t.x1 || ry < t.y0 || ry >= t.y1) continue;   // owned by another core
        const int32_t S = (int32_t)((int64_t)ry * g.W + rx + 1);
        atomicMin(g.labels + (int64_t)sy * g.out_pitch + sx, S);
        if (sx == rx && sy == ry && g.n_objects) atomicAdd(g.n_objects, 1);
    }
}

// unowned pixels (still INT32_MAX) become background; the mask follows
__global__ void k_stitch_final(int32_t *labels, uint8_t *mask, int64_t pitch, int W, int H) {
    const int64_t n = (int64_t)W * H;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        int32_t *p = labels + (int64_t)y * pitch + x;
        const int32_t v = *p == INT32_MAX ? 0 : *p;
        *p = v;
        if (mask) mask[(int64_t)y * pitch + x] = v ? 1 : 0;
    }
}

__global__ void k_stitch_init(int32_t *labels, int64_t pitch, int W, int H, int32_t *n_objects) {
    const int64_t n = (int64_t)W * H;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        labels[(int64_t)y * pitch + x] = INT32_MAX;
    }
    if (n_objects && blockIdx.x == 0 && threadIdx.x == 0) *n_objects = 0;
}

int grid_px(int64_t n, int n_cu) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, n_cu * 8)); }

}  // namespace

int launch_stitch_init(int32_t *labels, int64_t pitch, int W, int H, int32_t *n_objects, int n_cu, hipStream_t s) {
    hipLaunchKernelGGL(k_stitch_init, dim3(grid_px((int64_t)W * H, n_cu)), dim3(256), 0, s, labels, pitch, W, H,
                       n_objects);
    return hip_fail(hipGetLastError(), "k_stitch_init");
}

int launch_stitch(const StitchGroup &g, int n_cu, hipStream_t s) {
    if (g.n <= 0) return RT_OK;
    int64_t most = 1;
    for (int i = 0; i < g.n; ++i) most = std::max<int64_t>(most, (int64_t)g.t[i].ew * g.t[i].eh);
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((most + 255) / 256, std::max(1, n_cu * 8 / g.n)));
    hipLaunchKernelGGL(k_stitch, dim3(bx, g.n), dim3(256), 0, s, g);
    return hip_fail(hipGetLastError(), "k_stitch");
}

int launch_stitch_final(int32_t *labels, uint8_t *mask, int64_t pitch, int W, int H, int n_cu, hipStream_t s) {
    hipLaunchKernelGGL(k_stitch_final, dim3(grid_px((int64_t)W * H, n_cu)), dim3(256), 0, s, labels, mask, pitch, W,
                       H);
    return hip_fail(hipGetLastError(), "k_stitch_final");
}

}  // namespace rtseg
