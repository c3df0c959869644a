// Small element-wise kernels shared by several entry points: fills, and the
// area filter of rt_area_filter (labels produced by BWLabel).
#include "rt_internal.h"

namespace rtseg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
int launch_fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s) {
    if (!n) return RT_OK;
    int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(256), 0, s, p, v, n);
    return hip_fail(hipGetLastError(), "k_fill_i32");
}

// area filter on labels (root ids); area_scratch has w*h+1 entries
__global__ void k_area_zero(const int32_t *lab, int w, int h, int64_t pitch, int32_t *area) {
    int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        int l = lab[y * pitch + x];
        if (l > 0 && l <= n) area[l] = 0;
    }
}
__global__ void k_area_count(const int32_t *lab, int w, int h, int64_t pitch, int32_t *area) {
    int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        int l = lab[y * pitch + x];
        if (l > 0 && l <= n) atomicAdd(area + l, 1);
    }
}
__global__ void k_area_apply(const int32_t *lab, int32_t *out, uint8_t *mask, int w, int h, int64_t pitch,
                             const int32_t *area, int lo, int hi) {
    int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        int64_t o = y * pitch + x;
        int l = lab[o];
        int v = (l > 0 && l <= n && area[l] >= lo && area[l] <= hi) ? l : 0;
        out[o] = v;
        if (mask) mask[o] = v ? 1 : 0;
    }
}
int launch_area_filter(const int32_t *lab_in, int32_t *lab_out, uint8_t *mask_out, int w, int h, int64_t pitch,
                       int min_area, int max_area, int32_t *area, hipStream_t s) {
    int64_t n = (int64_t)w * h;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_area_zero, dim3(grid), dim3(256), 0, s, lab_in, w, h, pitch, area);
    hipLaunchKernelGGL(k_area_count, dim3(grid), dim3(256), 0, s, lab_in, w, h, pitch, area);
    hipLaunchKernelGGL(k_area_apply, dim3(grid), dim3(256), 0, s, lab_in, lab_out, mask_out, w, h, pitch, area,
                       min_area, max_area);
    return hip_fail(hipGetLastError(), "k_area");
}

}  // namespace rtseg
