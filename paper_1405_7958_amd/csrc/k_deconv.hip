// Colour deconvolution (Sec. 5.1, Ruifrok-Johnston stain separation):
// RGB bytes -> FP64 hematoxylin concentration c_H -> uint8 Hq.
//
// A per-call table T_k[v] = inv(M)[k][0] * (-ln((v+1)/256)) (3 x 256 FP64) is
// built on the device from the stain rows; each block stages it in LDS, and a
// pixel costs three LDS reads, two FP64 adds and one multiply-add pair (no
// contraction).  The kernel is a pure HBM stream: 3 bytes in, 1 byte out
// (+4 with the optional float c_H).  Each thread owns 16 consecutive pixels =
// three 16-byte loads and one 16-byte store.
#include "rt_internal.h"

namespace rtseg {

__global__ void k_deconv_lut(StainParams sp, double *__restrict__ lut) {
    double M[3][3];
    for (int i = 0; i < 3; ++i) {
        double n = sqrt(sp.rows[3 * i] * sp.rows[3 * i] + sp.rows[3 * i + 1] * sp.rows[3 * i + 1] +
                        sp.rows[3 * i + 2] * sp.rows[3 * i + 2]);
        for (int k = 0; k < 3; ++k) M[i][k] = n > 0.0 ? sp.rows[3 * i + k] / n : 0.0;
    }
    if (M[2][0] == 0.0 && M[2][1] == 0.0 && M[2][2] == 0.0) {
        double c0 = __dsub_rn(__dmul_rn(M[0][1], M[1][2]), __dmul_rn(M[0][2], M[1][1]));
        double c1 = __dsub_rn(__dmul_rn(M[0][2], M[1][0]), __dmul_rn(M[0][0], M[1][2]));
        double c2 = __dsub_rn(__dmul_rn(M[0][0], M[1][1]), __dmul_rn(M[0][1], M[1][0]));
        double n = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        M[2][0] = c0 / n;
        M[2][1] = c1 / n;
        M[2][2] = c2 / n;
    }
    // first column of inv(M) = first row of the cofactor matrix / det(M)
    double a0 = __dsub_rn(__dmul_rn(M[1][1], M[2][2]), __dmul_rn(M[1][2], M[2][1]));
    double a1 = -__dsub_rn(__dmul_rn(M[1][0], M[2][2]), __dmul_rn(M[1][2], M[2][0]));
    double a2 = __dsub_rn(__dmul_rn(M[1][0], M[2][1]), __dmul_rn(M[1][1], M[2][0]));
    double det = __dadd_rn(__dadd_rn(__dmul_rn(M[0][0], a0), __dmul_rn(M[0][1], a1)), __dmul_rn(M[0][2], a2));
    int v = threadIdx.x;
    double od = -log((double)(v + 1) / 256.0);
    lut[v] = __dmul_rn(a0 / det, od);
    lut[256 + v] = __dmul_rn(a1 / det, od);
    lut[512 + v] = __dmul_rn(a2 / det, od);
}

__device__ __forceinline__ uint8_t quantize(double c, double scale) {
    double q = floor(__dadd_rn(__dmul_rn(c, scale), 0.5));
    q = q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q);
    return (uint8_t)q;
}

__device__ __forceinline__ double chan(const double *T, uint32_t r, uint32_t g, uint32_t b) {
    return __dadd_rn(__dadd_rn(T[r], T[256 + g]), T[512 + b]);
}

// Fast path: dense images, 16 pixels per thread, grid-stride over groups.
template <bool WANT_CH, bool WANT_HIST>
__global__ __launch_bounds__(256) void k_deconv16(const double *__restrict__ lut, double scale,
                                                   const uint8_t *__restrict__ rgb, int64_t ngroups,
                                                   uint8_t *__restrict__ hq, float *__restrict__ ch,
                                                   uint32_t *__restrict__ hist) {
    __shared__ double T[768];
    __shared__ uint32_t H[256];
    for (int i = threadIdx.x; i < 768; i += blockDim.x) T[i] = lut[i];
    if (WANT_HIST) H[threadIdx.x] = 0;
    __syncthreads();
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *src = reinterpret_cast<const u32x4 *>(rgb);
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ngroups;
         g += (int64_t)gridDim.x * blockDim.x) {
        u32x4 v0 = __builtin_nontemporal_load(src + 3 * g);
        u32x4 v1 = __builtin_nontemporal_load(src + 3 * g + 1);
        u32x4 v2 = __builtin_nontemporal_load(src + 3 * g + 2);
        uint32_t wds[12] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x, v2.y, v2.z, v2.w};
        uint32_t out[4] = {0, 0, 0, 0};
        float cf[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            int b0 = 3 * p, b1 = 3 * p + 1, b2 = 3 * p + 2;
            uint32_t r = (wds[b0 >> 2] >> ((b0 & 3) * 8)) & 255u;
            uint32_t gg = (wds[b1 >> 2] >> ((b1 & 3) * 8)) & 255u;
            uint32_t b = (wds[b2 >> 2] >> ((b2 & 3) * 8)) & 255u;
            double c = chan(T, r, gg, b);
            uint32_t q = quantize(c, scale);
            out[p >> 2] |= q << ((p & 3) * 8);
            if (WANT_CH) cf[p] = (float)c;
            if (WANT_HIST) atomicAdd(&H[q], 1u);
        }
        reinterpret_cast<uint4 *>(hq)[g] = make_uint4(out[0], out[1], out[2], out[3]);
        if (WANT_CH) {
            float4 *cd = reinterpret_cast<float4 *>(ch) + 4 * g;
#pragma unroll
            for (int k = 0; k < 4; ++k) cd[k] = make_float4(cf[4 * k], cf[4 * k + 1], cf[4 * k + 2], cf[4 * k + 3]);
        }
    }
    if (WANT_HIST) {
        __syncthreads();
        if (H[threadIdx.x]) atomicAdd(&hist[threadIdx.x], H[threadIdx.x]);
    }
}

// Generic path: any pitch/alignment; pixels [first, w*h) in row-major order.
__global__ __launch_bounds__(256) void k_deconv_generic(const double *__restrict__ lut, double scale,
                                                         const uint8_t *__restrict__ rgb, int64_t rgb_pitch,
                                                         int w, int64_t first, int64_t npx,
                                                         uint8_t *__restrict__ hq, int64_t hq_pitch,
                                                         float *__restrict__ ch, int64_t ch_pitch,
                                                         uint32_t *__restrict__ hist) {
    __shared__ double T[768];
    __shared__ uint32_t H[256];
    for (int i = threadIdx.x; i < 768; i += blockDim.x) T[i] = lut[i];
    H[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = first + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npx;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        const uint8_t *px = rgb + y * rgb_pitch + 3 * x;
        double c = chan(T, px[0], px[1], px[2]);
        uint8_t q = quantize(c, scale);
        hq[y * hq_pitch + x] = q;
        if (ch) ch[y * ch_pitch + x] = (float)c;
        if (hist) atomicAdd(&H[q], 1u);
    }
    if (hist) {
        __syncthreads();
        if (H[threadIdx.x]) atomicAdd(&hist[threadIdx.x], H[threadIdx.x]);
    }
}

int launch_deconv_lut(const StainParams &sp, double *lut, int *, hipStream_t s) {
    hipLaunchKernelGGL(k_deconv_lut, dim3(1), dim3(256), 0, s, sp, lut);
    return hip_fail(hipGetLastError(), "k_deconv_lut");
}

int launch_deconv(const double *lut, double scale, const uint8_t *rgb, int64_t rgb_pitch, int w, int h,
                  float *ch, int64_t ch_pitch, uint8_t *hq, int64_t hq_pitch, uint8_t *, int64_t,
                  uint32_t *hist, int n_cu, hipStream_t s) {
    int64_t n = (int64_t)w * h;
    bool dense = rgb_pitch == 3LL * w && hq_pitch == w && (!ch || ch_pitch == w);
    bool aligned = ((uintptr_t)rgb % 16 == 0) && ((uintptr_t)hq % 16 == 0) && (!ch || (uintptr_t)ch % 16 == 0);
    int64_t first = 0;
    if (dense && aligned && n >= 16) {
        int64_t groups = n / 16;
        int64_t blocks = (groups + 255) / 256;
        int grid = (int)(blocks < (int64_t)n_cu * 8 ? blocks : (int64_t)n_cu * 8);
        if (ch) {
            if (hist)
                hipLaunchKernelGGL((k_deconv16<true, true>), dim3(grid), dim3(256), 0, s, lut, scale, rgb, groups, hq, ch, hist);
            else
                hipLaunchKernelGGL((k_deconv16<true, false>), dim3(grid), dim3(256), 0, s, lut, scale, rgb, groups, hq, ch, hist);
        } else {
            if (hist)
                hipLaunchKernelGGL((k_deconv16<false, true>), dim3(grid), dim3(256), 0, s, lut, scale, rgb, groups, hq, ch, hist);
            else
                hipLaunchKernelGGL((k_deconv16<false, false>), dim3(grid), dim3(256), 0, s, lut, scale, rgb, groups, hq, ch, hist);
        }
        int e = hip_fail(hipGetLastError(), "k_deconv16");
        if (e) return e;
        first = groups * 16;
    }
    if (first < n) {
        int64_t rem = n - first;
        int64_t blocks = (rem + 255) / 256;
        int grid = (int)(blocks < (int64_t)n_cu * 8 ? blocks : (int64_t)n_cu * 8);
        hipLaunchKernelGGL(k_deconv_generic, dim3(grid), dim3(256), 0, s, lut, scale, rgb, rgb_pitch, w, first, n,
                           hq, hq_pitch, ch, ch_pitch, hist);
        return hip_fail(hipGetLastError(), "k_deconv_generic");
    }
    return RT_OK;
}

}  // namespace rtseg
