// Colour deconvolution (Sec. 5.1, Ruifrok-Johnston stain separation):
// RGB bytes -> FP64 hematoxylin concentration c_H -> uint8 Hq.
//
// A per-call table T_k[v] = inv(M)[k][0] * (-ln((v+1)/256)) (3 x 256 FP64) is
// built on the device from the stain rows; each block stages it in LDS, and a
// pixel costs three LDS reads, two FP64 adds and one multiply-add pair (no
// contraction).  The kernel is a pure HBM stream: 3 bytes in, 1 byte out
// (+4 with the optional float c_H).
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

// Unit = a chunk of 4096 consecutive pixels (row-major) of one image; one
// 256-thread block handles a chunk, 16 pixels per thread.  Dense images with
// 16-byte aligned rows take three 16-byte loads and one 16-byte store per
// thread; others (pitched or unaligned) go pixel by pixel.  The block's
// histogram of a chunk is added to its image's histogram.
__device__ __forceinline__ int img_of(const DeconvImg *imgs, int n, int64_t u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].unit0 <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_deconv(const double *__restrict__ lut, double scale,
                                                 const DeconvImg *__restrict__ imgs, int n, int64_t total) {
    __shared__ double T[768];
    __shared__ uint32_t H[256];
    for (int i = threadIdx.x; i < 768; i += blockDim.x) T[i] = lut[i];
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    // the block's histogram runs over all its chunks of one image and is added
    // to one of HIST_COPIES copies of that image's histogram when the image
    // changes (spreads the global atomics over more addresses)
    const uint32_t copy = (blockIdx.x % HIST_COPIES) * 256u;
    int cur = -1;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        const int ii = img_of(imgs, n, u);
        if (ii != cur) {
            __syncthreads();
            if (cur >= 0 && imgs[cur].hist && H[threadIdx.x]) atomicAdd(&imgs[cur].hist[copy + threadIdx.x], H[threadIdx.x]);
            H[threadIdx.x] = 0;
            __syncthreads();
            cur = ii;
        }
        const DeconvImg im = imgs[ii];
        const int64_t npx = (int64_t)im.w * im.h;
        const int64_t p0 = (u - im.unit0) * DECONV_CHUNK + (int64_t)threadIdx.x * 16;
        const bool dense = im.rgb_pitch == 3LL * im.w && im.hq_pitch == im.w && (!im.ch || im.ch_pitch == im.w) &&
                           ((uintptr_t)im.rgb % 16 == 0) && ((uintptr_t)im.hq % 16 == 0) &&
                           (!im.ch || (uintptr_t)im.ch % 16 == 0);
        if (dense && p0 + 16 <= npx) {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(im.rgb + 3 * p0);
            u32x4 v0 = __builtin_nontemporal_load(src);
            u32x4 v1 = __builtin_nontemporal_load(src + 1);
            u32x4 v2 = __builtin_nontemporal_load(src + 2);
            uint32_t wds[12] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x, v2.y, v2.z, v2.w};
            uint32_t out[4] = {0, 0, 0, 0};
            float cf[16];
            // histogram by runs of equal values (background dominates, so one
            // LDS atomic covers most of a thread's 16 pixels)
            uint32_t run_q = 256u, run_n = 0u;
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const int b0 = 3 * p, b1 = 3 * p + 1, b2 = 3 * p + 2;
                const uint32_t r = (wds[b0 >> 2] >> ((b0 & 3) * 8)) & 255u;
                const uint32_t gg = (wds[b1 >> 2] >> ((b1 & 3) * 8)) & 255u;
                const uint32_t b = (wds[b2 >> 2] >> ((b2 & 3) * 8)) & 255u;
                const double c = chan(T, r, gg, b);
                const uint32_t q = quantize(c, scale);
                out[p >> 2] |= q << ((p & 3) * 8);
                cf[p] = (float)c;
                if (q == run_q) {
                    ++run_n;
                } else {
                    if (im.hist && run_n) atomicAdd(&H[run_q], run_n);
                    run_q = q;
                    run_n = 1u;
                }
            }
            if (im.hist && run_n) atomicAdd(&H[run_q], run_n);
            *reinterpret_cast<uint4 *>(im.hq + p0) = make_uint4(out[0], out[1], out[2], out[3]);
            if (im.ch) {
                float4 *cd = reinterpret_cast<float4 *>(im.ch + p0);
#pragma unroll
                for (int k = 0; k < 4; ++k) cd[k] = make_float4(cf[4 * k], cf[4 * k + 1], cf[4 * k + 2], cf[4 * k + 3]);
            }
        } else {
            for (int64_t p = p0; p < p0 + 16 && p < npx; ++p) {
                const int64_t y = p / im.w, x = p - y * im.w;
                const uint8_t *px = im.rgb + y * im.rgb_pitch + 3 * x;
                const double c = chan(T, px[0], px[1], px[2]);
                const uint8_t q = quantize(c, scale);
                im.hq[y * im.hq_pitch + x] = q;
                if (im.ch) im.ch[y * im.ch_pitch + x] = (float)c;
                if (im.hist) atomicAdd(&H[q], 1u);
            }
        }
    }
    __syncthreads();
    if (cur >= 0 && imgs[cur].hist && H[threadIdx.x]) atomicAdd(&imgs[cur].hist[copy + threadIdx.x], H[threadIdx.x]);
}

int launch_deconv_lut(const StainParams &sp, double *lut, hipStream_t s) {
    hipLaunchKernelGGL(k_deconv_lut, dim3(1), dim3(256), 0, s, sp, lut);
    return hip_fail(hipGetLastError(), "k_deconv_lut");
}

int launch_deconv(const double *lut, double scale, const DeconvImg *imgs_dev, int n, int64_t total, int n_cu,
                  hipStream_t s) {
    if (total <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>(total, (int64_t)n_cu * 8);
    hipLaunchKernelGGL(k_deconv, dim3(grid), dim3(256), 0, s, lut, scale, imgs_dev, n, total);
    return hip_fail(hipGetLastError(), "k_deconv");
}

}  // namespace rtseg
