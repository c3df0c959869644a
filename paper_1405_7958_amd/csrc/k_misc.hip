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

__global__ void k_zero_u8(uint8_t *p, int64_t pitch, int w, int h) {
    const int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / w, x = i - y * w;
        p[y * pitch + x] = 0;
    }
}
int launch_zero_u8(uint8_t *p, int64_t pitch, int w, int h, hipStream_t s) {
    const int64_t n = (int64_t)w * h;
    if (n <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_u8, dim3(grid), dim3(256), 0, s, p, pitch, w, h);
    return hip_fail(hipGetLastError(), "k_zero_u8");
}

__global__ void k_surrogate_maps(const float *pf, const float *ps, int64_t n, uint8_t *fg, uint8_t *seeds,
                                 int32_t *counts) {
    int c[4] = {0, 0, 0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float f = pf[i], q = ps[i];
        fg[i] = f >= 0.5f ? 1 : 0;
        seeds[i] = q >= 0.5f ? 1 : 0;
        c[0] += f >= 0.25f;
        c[1] += (f >= 0.25f && f < 0.75f);
        c[2] += q >= 0.25f;
        c[3] += (q >= 0.25f && q < 0.75f);
    }
    // wave sums, then block sums in LDS: one atomic per block and counter
    __shared__ int red[4][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int v = c[k];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (v) atomicAdd(counts + threadIdx.x, v);
    }
}
int launch_surrogate_maps(const float *p_fg, const float *p_seed, int w, int h, uint8_t *fg, uint8_t *seeds,
                          int32_t *counts, hipStream_t s) {
    const int64_t n = (int64_t)w * h;
    if (n <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_surrogate_maps, dim3(grid), dim3(256), 0, s, p_fg, p_seed, n, fg, seeds, counts);
    return hip_fail(hipGetLastError(), "k_surrogate_maps");
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
