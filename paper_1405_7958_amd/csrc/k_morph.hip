// Pre-processing operations the paper lists beside the segmentation
// (Sec. 5.1: Morphological Open, RBC detection; the ReconToNuclei marker):
// grey erosion / dilation by a flat disk, the frame marker, the top-hat
// threshold and the RBC redness maps.  The reconstructions they feed run on
// the reconstruction round kernel.
//
// Erosion / dilation: one 256-thread block per 64 x 32 output tile.  The
// tile and an r-pixel halo are staged in LDS with 16-byte loads where the
// row allows it (pixels outside the image take the operator's neutral value,
// 255 for the minimum and 0 for the maximum, so they never win); each thread
// then produces one column of 8 outputs, walking the disk as one horizontal
// span per row offset.  The disk's spans come from the host.
#include "rt_internal.h"

namespace rtseg {

namespace {

constexpr int MTW = 64, MTH = 32;   // output tile
constexpr int MROWS = 8;            // outputs per thread (a column of 8)

template <bool ERODE>
__global__ __launch_bounds__(256) void k_morph(MorphArgs a) {
    extern __shared__ uint8_t t[];
    const int r = a.radius;
    const int tw = MTW + 2 * r, th = MTH + 2 * r;
    const int tiles_x = (a.w + MTW - 1) / MTW, tiles_y = (a.h + MTH - 1) / MTH;
    const uint8_t neutral = ERODE ? 255 : 0;
    for (int tile = blockIdx.x; tile < tiles_x * tiles_y; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * MTW - r, y0 = (tile / tiles_x) * MTH - r;
        // stage: one byte per thread step (rows are short; the loads coalesce along the row)
        for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
            const int ly = i / tw, lx = i - ly * tw;
            const int x = x0 + lx, y = y0 + ly;
            t[i] = (x >= 0 && x < a.w && y >= 0 && y < a.h) ? a.in[(int64_t)y * a.in_pitch + x] : neutral;
        }
        __syncthreads();
        const int cx = threadIdx.x % MTW, ry = (threadIdx.x / MTW) * MROWS;
        int acc[MROWS];
#pragma unroll
        for (int k = 0; k < MROWS; ++k) acc[k] = neutral;
        // row offset dy: span [-s, s]; the block row ly = ry + k + r + dy
        for (int dy = -r; dy <= r; ++dy) {
            const int s = a.span[dy + r];
            for (int dx = -s; dx <= s; ++dx) {
                const int lx = cx + r + dx;
#pragma unroll
                for (int k = 0; k < MROWS; ++k) {
                    const int v = t[(ry + k + r + dy) * tw + lx];
                    acc[k] = ERODE ? min(acc[k], v) : max(acc[k], v);
                }
            }
        }
        const int ox = x0 + r + cx;
#pragma unroll
        for (int k = 0; k < MROWS; ++k) {
            const int oy = y0 + r + ry + k;
            if (ox < a.w && oy < a.h) a.out[(int64_t)oy * a.out_pitch + ox] = (uint8_t)acc[k];
        }
        __syncthreads();
    }
}

// R = Hq on the one-pixel frame, 0 inside (the plain ReconToNuclei marker)
__global__ void k_frame_marker(const uint8_t *hq, int64_t hq_pitch, uint8_t *r, int64_t r_pitch, int w, int h) {
    const int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / w), x = (int)(i - (int64_t)y * w);
        const bool frame = x == 0 || y == 0 || x == w - 1 || y == h - 1;
        r[(int64_t)y * r_pitch + x] = frame ? hq[(int64_t)y * hq_pitch + x] : 0;
    }
}

// F0 = [Hq - R >= t]
__global__ void k_tophat(const uint8_t *hq, int64_t hq_pitch, const uint8_t *r, int64_t r_pitch, uint8_t *f0,
                         int64_t f0_pitch, int w, int h, int t) {
    const int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / w), x = (int)(i - (int64_t)y * w);
        const int d = (int)hq[(int64_t)y * hq_pitch + x] - (int)r[(int64_t)y * r_pitch + x];
        f0[(int64_t)y * f0_pitch + x] = d >= t ? 1 : 0;
    }
}

// redness 2R - G - B: weak = [>= t_weak] (the mask), strong = weak and
// [>= t_strong] (the marker), as 0/1 bytes
__global__ void k_rbc_maps(const uint8_t *rgb, int64_t rgb_pitch, int w, int h, int t_strong, int t_weak,
                           uint8_t *marker, uint8_t *mask, int64_t pitch) {
    const int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / w), x = (int)(i - (int64_t)y * w);
        const uint8_t *p = rgb + (int64_t)y * rgb_pitch + 3 * x;
        const int red = 2 * (int)p[0] - (int)p[1] - (int)p[2];
        const bool weak = red >= t_weak;
        mask[(int64_t)y * pitch + x] = weak ? 1 : 0;
        marker[(int64_t)y * pitch + x] = (weak && red >= t_strong) ? 1 : 0;
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

size_t morph_lds_bytes(int radius) { return (size_t)(MTW + 2 * radius) * (MTH + 2 * radius); }

int launch_morph(const MorphArgs &a, bool erode, int n_cu, hipStream_t s) {
    if (a.radius < 0 || a.radius > RT_MORPH_MAX_RADIUS) {
        set_error("morphology: radius %d outside 0..%d", a.radius, RT_MORPH_MAX_RADIUS);
        return RT_EINVAL;
    }
    const int tiles = ((a.w + MTW - 1) / MTW) * ((a.h + MTH - 1) / MTH);
    const int grid = std::max(1, std::min(tiles, n_cu * 16));
    const size_t lds = morph_lds_bytes(a.radius);
    if (erode)
        hipLaunchKernelGGL(k_morph<true>, dim3(grid), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(k_morph<false>, dim3(grid), dim3(256), lds, s, a);
    return hip_fail(hipGetLastError(), "k_morph");
}

int launch_frame_marker(const uint8_t *hq, int64_t hq_pitch, uint8_t *r, int64_t r_pitch, int w, int h,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_frame_marker, dim3(grid_for((int64_t)w * h)), dim3(256), 0, s, hq, hq_pitch, r, r_pitch, w,
                       h);
    return hip_fail(hipGetLastError(), "k_frame_marker");
}

int launch_tophat(const uint8_t *hq, int64_t hq_pitch, const uint8_t *r, int64_t r_pitch, uint8_t *f0,
                  int64_t f0_pitch, int w, int h, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_tophat, dim3(grid_for((int64_t)w * h)), dim3(256), 0, s, hq, hq_pitch, r, r_pitch, f0,
                       f0_pitch, w, h, t);
    return hip_fail(hipGetLastError(), "k_tophat");
}

int launch_rbc_maps(const uint8_t *rgb, int64_t rgb_pitch, int w, int h, int t_strong, int t_weak, uint8_t *marker,
                    uint8_t *mask, int64_t pitch, hipStream_t s) {
    hipLaunchKernelGGL(k_rbc_maps, dim3(grid_for((int64_t)w * h)), dim3(256), 0, s, rgb, rgb_pitch, w, h, t_strong,
                       t_weak, marker, mask, pitch);
    return hip_fail(hipGetLastError(), "k_rbc_maps");
}

}  // namespace rtseg
