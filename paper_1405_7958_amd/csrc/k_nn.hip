// Layer kernels of the U-Net surrogate on the CDNA4 matrix cores.
//
// Every contraction is an implicit GEMM fed straight from NHWC bfloat16
// tensors into v_mfma_f32_16x16x32_bf16 (FP32 accumulation):
//   conv3 forward   M = pixels, N = co, K = 9 ci   (A: 8 consecutive channels
//                   of one tap of one pixel per lane, B: weights [co][9][ci])
//   conv3 dgrad     the same kernel with the tap offsets negated, N = ci and
//                   the weights transposed to [ci][9][co]
//   up2 forward     M = input pixels of one output parity (a, b), N = co, K = ci
//   up2 dgrad       M = input pixels, N = ci, K = 4 co (the four output pixels)
//   weight grads    M = output channels, N = (tap, ci), K = pixels, split over
//                   pixel chunks with float atomics
// A wave computes a 32 x (16 TN) tile of the output (two 16-row M tiles that
// share every B fragment); a 256-thread block holds four waves on adjacent
// pixel runs, so a block's A loads of neighbouring taps hit the same lines.
#include <algorithm>
#include <cmath>

#include "nn_internal.h"
#include "rt_internal.h"

namespace rtseg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

union V8 {
    uint4 u;
    bf16x8 v;
    bf16_t h[8];
};

// round to nearest even (NaN -> quiet NaN)
__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const bf16_t *p) {
    V8 t;
    t.u = *reinterpret_cast<const uint4 *>(p);
    return t.v;
}
__device__ __forceinline__ bf16x8 zero8() {
    V8 t;
    t.u = make_uint4(0, 0, 0, 0);
    return t.v;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// conv3 forward / dgrad
// ---------------------------------------------------------------------------
struct Conv3K {
    const bf16_t *x0, *x1;   // K-dimension channel sources (x1 nullable)
    int c0, c1;
    int n, h, w;
    int sgn;                 // +1: forward taps, -1: transposed taps
    const bf16_t *wk;        // [nout][9][c0 + c1]
    int nout;
    const float *bias;
    int relu;
    bf16_t *y;               // forward: bf16 output (nullable)
    float *yf;               // forward: f32 output (nullable)
    float *d0, *d1;          // dgrad: f32 outputs split at `split`
    int split;
    int dgrad;
};

template <int TN, int TM>
__global__ __launch_bounds__(256) void k_conv3(Conv3K a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)a.n * a.h * a.w;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * (16 * TM);
    if (base >= P) return;
    const int cin = a.c0 + a.c1;
    const int K = 9 * cin;
    const int r = lane & 15, kg = lane >> 4;
    const int hw = a.h * a.w;
    int img[TM], py[TM], px[TM];
    bool valid[TM];
#pragma unroll
    for (int mt = 0; mt < TM; ++mt) {
        const int64_t p = base + mt * 16 + r;
        valid[mt] = p < P;
        const int64_t pp = valid[mt] ? p : 0;
        img[mt] = (int)(pp / hw);
        const int rem = (int)(pp - (int64_t)img[mt] * hw);
        py[mt] = rem / a.w;
        px[mt] = rem - py[mt] * a.w;
    }
    f32x4 acc[TM][TN];
#pragma unroll
    for (int mt = 0; mt < TM; ++mt)
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < K; kb += 32) {
        const int k0 = kb + kg * 8;
        bf16x8 A[TM], B[TN];
        if (k0 < K) {
            const int tap = k0 / cin;
            const int ci = k0 - tap * cin;
            const int dy = a.sgn * (tap / 3 - 1), dx = a.sgn * (tap % 3 - 1);
#pragma unroll
            for (int mt = 0; mt < TM; ++mt) {
                const int sy = py[mt] + dy, sx = px[mt] + dx;
                if (valid[mt] && sy >= 0 && sy < a.h && sx >= 0 && sx < a.w) {
                    const int64_t sp = ((int64_t)img[mt] * a.h + sy) * a.w + sx;
                    A[mt] = ci < a.c0 ? load8(a.x0 + sp * a.c0 + ci) : load8(a.x1 + sp * a.c1 + (ci - a.c0));
                } else {
                    A[mt] = zero8();
                }
            }
#pragma unroll
            for (int t = 0; t < TN; ++t) B[t] = load8(a.wk + (int64_t)(t * 16 + r) * K + k0);
        } else {
#pragma unroll
            for (int mt = 0; mt < TM; ++mt) A[mt] = zero8();
#pragma unroll
            for (int t = 0; t < TN; ++t) B[t] = zero8();
        }
#pragma unroll
        for (int mt = 0; mt < TM; ++mt)
#pragma unroll
            for (int t = 0; t < TN; ++t) acc[mt][t] = mfma(A[mt], B[t], acc[mt][t]);
    }
    // D layout: lane holds rows 4*kg + e of column r
#pragma unroll
    for (int mt = 0; mt < TM; ++mt) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = base + mt * 16 + kg * 4 + e;
            if (p >= P) continue;
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                const int nn = t * 16 + r;
                float v = acc[mt][t][e];
                if (!a.dgrad) {
                    v += a.bias[nn];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    if (a.y) a.y[p * a.nout + nn] = f2bf(v);
                    if (a.yf) a.yf[p * a.nout + nn] = v;
                } else if (nn < a.split) {
                    a.d0[p * a.split + nn] = v;
                } else {
                    a.d1[p * (a.nout - a.split) + (nn - a.split)] = v;
                }
            }
        }
    }
}

// The same contraction with the input neighbourhood staged in LDS: a
// workgroup covers 4*RW output rows x 32 columns of one image; its
// (4*RW + 2) x 34 x cin input patch (zeros outside the image) is loaded once
// with 16-byte coalesced reads, and every tap's A fragment is then read from
// LDS instead of from L1/L2 nine times over.  Wave w computes rows
// w*RW .. w*RW+RW-1, two 16-pixel M tiles per row.
constexpr int PW = 34;   // patch width: 32 columns + halo

template <int TN, int RW>
__global__ __launch_bounds__(256) void k_conv3_lds(Conv3K a) {
    extern __shared__ __align__(16) bf16_t patch[];
    constexpr int TM = 2 * RW;
    constexpr int TH = 4 * RW;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int cin = a.c0 + a.c1;
    const int K = 9 * cin;
    const int bx = blockIdx.x, by = blockIdx.y, img = blockIdx.z;
    const int x0 = bx * 32, y0 = by * TH;
    // ---- stage the input patch
    const int c8 = cin / 8;
    const int chunks = (TH + 2) * PW * c8;
    for (int q = threadIdx.x; q < chunks; q += 256) {
        const int cc = q % c8;
        const int pix = q / c8;
        const int pc = pix % PW, pr = pix / PW;
        const int gy = y0 + pr - 1, gx = x0 + pc - 1;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < a.h && gx >= 0 && gx < a.w) {
            const int64_t sp = ((int64_t)img * a.h + gy) * a.w + gx;
            const int ci = cc * 8;
            v = ci < a.c0 ? *reinterpret_cast<const uint4 *>(a.x0 + sp * a.c0 + ci)
                          : *reinterpret_cast<const uint4 *>(a.x1 + sp * a.c1 + (ci - a.c0));
        }
        *reinterpret_cast<uint4 *>(patch + (int64_t)pix * cin + cc * 8) = v;
    }
    __syncthreads();
    const int r = lane & 15, kg = lane >> 4;
    f32x4 acc[TM][TN];
#pragma unroll
    for (int mt = 0; mt < TM; ++mt)
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < K; kb += 32) {
        const int k0 = kb + kg * 8;
        bf16x8 A[TM], B[TN];
        if (k0 < K) {
            const int tap = k0 / cin;
            const int ci = k0 - tap * cin;
            const int dy = a.sgn * (tap / 3 - 1), dx = a.sgn * (tap % 3 - 1);
#pragma unroll
            for (int mt = 0; mt < TM; ++mt) {
                const int row = wave * RW + (mt >> 1) + 1 + dy;
                const int col = (mt & 1) * 16 + r + 1 + dx;
                A[mt] = load8(patch + (row * PW + col) * cin + ci);
            }
#pragma unroll
            for (int t = 0; t < TN; ++t) B[t] = load8(a.wk + (int64_t)(t * 16 + r) * K + k0);
        } else {
#pragma unroll
            for (int mt = 0; mt < TM; ++mt) A[mt] = zero8();
#pragma unroll
            for (int t = 0; t < TN; ++t) B[t] = zero8();
        }
#pragma unroll
        for (int mt = 0; mt < TM; ++mt)
#pragma unroll
            for (int t = 0; t < TN; ++t) acc[mt][t] = mfma(A[mt], B[t], acc[mt][t]);
    }
#pragma unroll
    for (int mt = 0; mt < TM; ++mt) {
        const int y = y0 + wave * RW + (mt >> 1);
        if (y >= a.h) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = x0 + (mt & 1) * 16 + kg * 4 + e;
            if (x >= a.w) continue;
            const int64_t p = ((int64_t)img * a.h + y) * a.w + x;
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                const int nn = t * 16 + r;
                float v = acc[mt][t][e];
                if (!a.dgrad) {
                    v += a.bias[nn];
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    if (a.y) a.y[p * a.nout + nn] = f2bf(v);
                    if (a.yf) a.yf[p * a.nout + nn] = v;
                } else if (nn < a.split) {
                    a.d0[p * a.split + nn] = v;
                } else {
                    a.d1[p * (a.nout - a.split) + (nn - a.split)] = v;
                }
            }
        }
    }
}

template <int TN, int RW>
static void launch_conv3_lds(const Conv3K &a, hipStream_t s) {
    const int cin = a.c0 + a.c1;
    const size_t lds = (size_t)(4 * RW + 2) * PW * cin * sizeof(bf16_t);
    static bool set = false;
    if (!set) {
        (void)hipFuncSetAttribute((const void *)k_conv3_lds<TN, RW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)((4 * RW + 2) * PW * 128 * sizeof(bf16_t)));
        set = true;
    }
    const dim3 grid((unsigned)((a.w + 31) / 32), (unsigned)((a.h + 4 * RW - 1) / (4 * RW)), (unsigned)a.n);
    hipLaunchKernelGGL((k_conv3_lds<TN, RW>), grid, dim3(256), lds, s, a);
}

static int launch_conv3(const Conv3K &a, hipStream_t s) {
    if (a.nout % 16 || a.nout > 128 || a.nout < 16 || (a.c0 % 8) || (a.c1 % 8)) {
        set_error("nn conv3: unsupported channel counts (in %d+%d, out %d)", a.c0, a.c1, a.nout);
        return RT_EINVAL;
    }
    const int64_t P = (int64_t)a.n * a.h * a.w;
    if (P <= 0) return RT_OK;
    // a wave computes 16*TM pixels x nout channels; wider outputs take more
    // pixels per wave so that each weight fragment feeds more matrix ops
    const int tn = a.nout / 16;
    const int cin = a.c0 + a.c1;
    if (cin <= 128 && a.n <= 65535) {
        switch (tn) {
            case 1: launch_conv3_lds<1, 1>(a, s); break;
            case 2: launch_conv3_lds<2, 1>(a, s); break;
            case 4: launch_conv3_lds<4, 2>(a, s); break;
            case 8: launch_conv3_lds<8, 2>(a, s); break;
            default: goto direct;
        }
        return hip_fail(hipGetLastError(), "k_conv3_lds");
    }
direct:
    const int tm = tn >= 4 ? 4 : 2;
    const dim3 grid((unsigned)((P + 64 * tm - 1) / (64 * tm)));
    switch (tn) {
        case 1: hipLaunchKernelGGL((k_conv3<1, 2>), grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_conv3<2, 2>), grid, dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_conv3<3, 2>), grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_conv3<4, 4>), grid, dim3(256), 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_conv3<5, 4>), grid, dim3(256), 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_conv3<6, 4>), grid, dim3(256), 0, s, a); break;
        case 7: hipLaunchKernelGGL((k_conv3<7, 4>), grid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((k_conv3<8, 4>), grid, dim3(256), 0, s, a); break;
    }
    return hip_fail(hipGetLastError(), "k_conv3");
}

int nn_conv3_fwd(const bf16_t *x0, int c0, const bf16_t *x1, int c1, int n, int h, int w, const bf16_t *wk,
                 const float *bias, int co, int relu, bf16_t *y, float *yf, hipStream_t s) {
    Conv3K a{};
    a.x0 = x0;
    a.x1 = x1;
    a.c0 = c0;
    a.c1 = x1 ? c1 : 0;
    a.n = n;
    a.h = h;
    a.w = w;
    a.sgn = 1;
    a.wk = wk;
    a.nout = co;
    a.bias = bias;
    a.relu = relu;
    a.y = y;
    a.yf = yf;
    return launch_conv3(a, s);
}

int nn_conv3_dgrad(const bf16_t *g, int co, int n, int h, int w, const bf16_t *wt, int ci, int c0, float *dx0,
                   float *dx1, hipStream_t s) {
    Conv3K a{};
    a.x0 = g;
    a.c0 = co;
    a.n = n;
    a.h = h;
    a.w = w;
    a.sgn = -1;
    a.wk = wt;
    a.nout = ci;
    a.dgrad = 1;
    a.d0 = dx0;
    a.d1 = dx1;
    a.split = c0;
    if (c0 % 16 || (c0 < ci && !dx1)) {
        set_error("nn conv3 dgrad: bad split %d of %d", c0, ci);
        return RT_EINVAL;
    }
    return launch_conv3(a, s);
}

// ---------------------------------------------------------------------------
// up2 forward / dgrad
// ---------------------------------------------------------------------------
struct Up2K {
    const bf16_t *x;   // forward: x (n, h, w, cx); dgrad: g (n, 2h, 2w, cx)
    int cx;
    int n, h, w;       // input grid
    const bf16_t *wk;  // forward: [4][nout][cx]; dgrad: [nout][4][cx]
    int nout;
    int dgrad;
    const float *bias;
    bf16_t *y;
    float *yf;
    float *dx;
};

template <int TN>
__global__ __launch_bounds__(256) void k_up2(Up2K a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)a.n * a.h * a.w;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 32;
    if (base >= P) return;
    const int ab = blockIdx.y;   // forward: output parity of this launch slice
    const int K = a.dgrad ? 4 * a.cx : a.cx;
    const int r = lane & 15, kg = lane >> 4;
    const int hw = a.h * a.w;
    int img[2], py[2], px[2];
    bool valid[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int64_t p = base + mt * 16 + r;
        valid[mt] = p < P;
        const int64_t pp = valid[mt] ? p : 0;
        img[mt] = (int)(pp / hw);
        const int rem = (int)(pp - (int64_t)img[mt] * hw);
        py[mt] = rem / a.w;
        px[mt] = rem - py[mt] * a.w;
    }
    f32x4 acc[2][TN];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int H2 = 2 * a.h, W2 = 2 * a.w;
    for (int kb = 0; kb < K; kb += 32) {
        const int k0 = kb + kg * 8;
        bf16x8 A[2], B[TN];
        if (k0 < K) {
            if (!a.dgrad) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const int64_t p = base + mt * 16 + r;
                    A[mt] = valid[mt] ? load8(a.x + p * a.cx + k0) : zero8();
                }
#pragma unroll
                for (int t = 0; t < TN; ++t) B[t] = load8(a.wk + ((int64_t)ab * a.nout + t * 16 + r) * K + k0);
            } else {
                const int q = k0 / a.cx;
                const int co = k0 - q * a.cx;
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const int64_t op = ((int64_t)img[mt] * H2 + 2 * py[mt] + (q >> 1)) * W2 + 2 * px[mt] + (q & 1);
                    A[mt] = valid[mt] ? load8(a.x + op * a.cx + co) : zero8();
                }
#pragma unroll
                for (int t = 0; t < TN; ++t) B[t] = load8(a.wk + (int64_t)(t * 16 + r) * K + k0);
            }
        } else {
            A[0] = A[1] = zero8();
#pragma unroll
            for (int t = 0; t < TN; ++t) B[t] = zero8();
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int t = 0; t < TN; ++t) acc[mt][t] = mfma(A[mt], B[t], acc[mt][t]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = base + mt * 16 + kg * 4 + e;
            if (p >= P) continue;
            const int im = (int)(p / hw);
            const int rem = (int)(p - (int64_t)im * hw);
            const int i = rem / a.w, j = rem - (rem / a.w) * a.w;
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                const int nn = t * 16 + r;
                const float v = acc[mt][t][e];
                if (!a.dgrad) {
                    const int64_t op = ((int64_t)im * H2 + 2 * i + (ab >> 1)) * W2 + 2 * j + (ab & 1);
                    const float o = v + a.bias[nn];
                    if (a.y) a.y[op * a.nout + nn] = f2bf(o);
                    if (a.yf) a.yf[op * a.nout + nn] = o;
                } else {
                    a.dx[p * a.nout + nn] = v;
                }
            }
        }
    }
}

static int launch_up2(const Up2K &a, hipStream_t s) {
    if (a.nout % 16 || a.nout > 128 || a.nout < 16 || a.cx % 8) {
        set_error("nn up2: unsupported channel counts (in %d, out %d)", a.cx, a.nout);
        return RT_EINVAL;
    }
    const int64_t P = (int64_t)a.n * a.h * a.w;
    if (P <= 0) return RT_OK;
    const dim3 grid((unsigned)((P + 127) / 128), a.dgrad ? 1 : 4);
    switch (a.nout / 16) {
        case 1: hipLaunchKernelGGL(k_up2<1>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_up2<2>, grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_up2<4>, grid, dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_up2<8>, grid, dim3(256), 0, s, a); break;
        default:
            set_error("nn up2: output channels must be 16, 32, 64 or 128");
            return RT_EINVAL;
    }
    return hip_fail(hipGetLastError(), "k_up2");
}

int nn_up2_fwd(const bf16_t *x, int ci, int n, int h, int w, const bf16_t *uf, const float *bias, int co, bf16_t *y,
               float *yf, hipStream_t s) {
    Up2K a{};
    a.x = x;
    a.cx = ci;
    a.n = n;
    a.h = h;
    a.w = w;
    a.wk = uf;
    a.nout = co;
    a.bias = bias;
    a.y = y;
    a.yf = yf;
    return launch_up2(a, s);
}

int nn_up2_dgrad(const bf16_t *g, int co, int n, int h, int w, const bf16_t *ut, int ci, float *dx, hipStream_t s) {
    Up2K a{};
    a.x = g;
    a.cx = co;
    a.n = n;
    a.h = h;
    a.w = w;
    a.wk = ut;
    a.nout = ci;
    a.dgrad = 1;
    a.dx = dx;
    return launch_up2(a, s);
}

// ---------------------------------------------------------------------------
// weight gradients: M = output rows of dw, N = its columns, K = pixels
// ---------------------------------------------------------------------------
struct WgradK {
    const bf16_t *x0, *x1;   // conv3: the layer input (concat); up2: the layer input
    int c0, c1;
    const bf16_t *g;         // gradient of the layer output (pre-activation), bf16
    int cg;
    int n, h, w;             // K pixel grid (conv3: image; up2: input)
    int M, N;
    float *dw;               // [M][N], accumulated
    int64_t chunk;           // pixels per block
};

// MODE 0: conv3  dw[co][tap*cin + ci]:  A(co, p) = g[p][co],  B(p, (tap, ci)) = x[p + off(tap)][ci]
// MODE 1: up2    dw[ci][ab*co + co]:    A(ci, p) = x[p][ci],  B(p, (ab, co)) = g[out(p, ab)][co]
template <int MODE>
__global__ __launch_bounds__(64) void k_wgrad(WgradK a) {
    const int lane = threadIdx.x;
    const int r = lane & 15, kg = lane >> 4;
    const int mblocks = a.M / 16;
    const int mb = blockIdx.x % mblocks, nb = blockIdx.x / mblocks;
    const int64_t P = (int64_t)a.n * a.h * a.w;
    const int64_t p0 = (int64_t)blockIdx.y * a.chunk;
    const int64_t p1 = p0 + a.chunk < P ? p0 + a.chunk : P;
    const int hw = a.h * a.w;
    const int m = mb * 16 + r;
    const int cin = a.c0 + a.c1;
    int ncol[4], q[4], ch[4];
    bool nok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        ncol[t] = nb * 64 + t * 16 + r;
        nok[t] = ncol[t] < a.N;
        const int div = MODE == 0 ? cin : a.cg;
        q[t] = nok[t] ? ncol[t] / div : 0;       // conv3: tap; up2: output parity
        ch[t] = nok[t] ? ncol[t] - q[t] * div : 0;
    }
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t kb = p0; kb < p1; kb += 32) {
        V8 A, B[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t p = kb + kg * 8 + e;
            if (p < p1) {
                const int im = (int)(p / hw);
                const int rem = (int)(p - (int64_t)im * hw);
                const int y = rem / a.w, x = rem - (rem / a.w) * a.w;
                if (MODE == 0) {
                    A.h[e] = a.g[p * a.cg + m];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int sy = y + q[t] / 3 - 1, sx = x + q[t] % 3 - 1;
                        bf16_t v = 0;
                        if (nok[t] && sy >= 0 && sy < a.h && sx >= 0 && sx < a.w) {
                            const int64_t sp = ((int64_t)im * a.h + sy) * a.w + sx;
                            v = ch[t] < a.c0 ? a.x0[sp * a.c0 + ch[t]] : a.x1[sp * a.c1 + ch[t] - a.c0];
                        }
                        B[t].h[e] = v;
                    }
                } else {
                    A.h[e] = a.x0[p * a.c0 + m];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int64_t op = ((int64_t)im * 2 * a.h + 2 * y + (q[t] >> 1)) * (2 * a.w) + 2 * x + (q[t] & 1);
                        B[t].h[e] = nok[t] ? a.g[op * a.cg + ch[t]] : (bf16_t)0;
                    }
                }
            } else {
                A.h[e] = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) B[t].h[e] = 0;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mfma(A.v, B[t].v, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (!nok[t]) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = mb * 16 + kg * 4 + e;
            atomicAdd(a.dw + (int64_t)row * a.N + ncol[t], acc[t][e]);
        }
    }
}

static int launch_wgrad(WgradK a, int mode, hipStream_t s) {
    if (a.M % 16) {
        set_error("nn wgrad: rows must be a multiple of 16 (got %d)", a.M);
        return RT_EINVAL;
    }
    const int64_t P = (int64_t)a.n * a.h * a.w;
    if (P <= 0) return RT_OK;
    const int blocks = (a.M / 16) * ((a.N + 63) / 64);
    // about 8192 waves in all, at least 256 pixels per chunk
    int64_t chunks = std::max<int64_t>(1, std::min<int64_t>((P + 255) / 256, 8192 / blocks));
    a.chunk = ((P + chunks - 1) / chunks + 31) / 32 * 32;
    chunks = (P + a.chunk - 1) / a.chunk;
    const dim3 grid((unsigned)blocks, (unsigned)chunks);
    if (mode == 0)
        hipLaunchKernelGGL(k_wgrad<0>, grid, dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(k_wgrad<1>, grid, dim3(64), 0, s, a);
    return hip_fail(hipGetLastError(), "k_wgrad");
}

int nn_conv3_wgrad(const bf16_t *x0, int c0, const bf16_t *x1, int c1, const bf16_t *g, int co, int n, int h, int w,
                   float *dw, hipStream_t s) {
    WgradK a{};
    a.x0 = x0;
    a.x1 = x1;
    a.c0 = c0;
    a.c1 = x1 ? c1 : 0;
    a.g = g;
    a.cg = co;
    a.n = n;
    a.h = h;
    a.w = w;
    a.M = co;
    a.N = 9 * (a.c0 + a.c1);
    a.dw = dw;
    return launch_wgrad(a, 0, s);
}

int nn_up2_wgrad(const bf16_t *x, int ci, const bf16_t *g, int co, int n, int h, int w, float *dw, hipStream_t s) {
    WgradK a{};
    a.x0 = x;
    a.c0 = ci;
    a.g = g;
    a.cg = co;
    a.n = n;
    a.h = h;
    a.w = w;
    a.M = ci;
    a.N = 4 * co;
    a.dw = dw;
    return launch_wgrad(a, 1, s);
}

// ---------------------------------------------------------------------------
// element-wise layers
// ---------------------------------------------------------------------------
__global__ void k_colsum(const bf16_t *g, int c, int64_t pixels, int64_t chunk, float *db) {
    __shared__ float red[256];
    const int groups = 256 / c;
    const int ch = threadIdx.x % c, grp = threadIdx.x / c;
    float sum = 0.f;
    if (grp < groups) {
        const int64_t p0 = (int64_t)blockIdx.x * chunk;
        const int64_t p1 = p0 + chunk < pixels ? p0 + chunk : pixels;
        for (int64_t p = p0 + grp; p < p1; p += groups) sum += bf2f(g[p * c + ch]);
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x < c) {
        float t = 0.f;
        for (int k = 0; k < groups; ++k) t += red[k * c + threadIdx.x];
        atomicAdd(db + threadIdx.x, t);
    }
}

int nn_colsum(const bf16_t *g, int c, int64_t pixels, float *db, hipStream_t s) {
    if (c < 1 || c > 256 || 256 % c) {
        set_error("nn colsum: channels must divide 256");
        return RT_EINVAL;
    }
    if (pixels <= 0) return RT_OK;
    const int64_t chunk = 4096;
    const int64_t blocks = (pixels + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)blocks), dim3(256), 0, s, g, c, pixels, chunk, db);
    return hip_fail(hipGetLastError(), "k_colsum");
}

__global__ void k_relu_bwd(const float *dy, const bf16_t *y, int64_t count, bf16_t *g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        float v = dy[i];
        if (y && !(bf2f(y[i]) > 0.f)) v = 0.f;
        g[i] = f2bf(v);
    }
}

int nn_relu_bwd(const float *dy, const bf16_t *y, int64_t count, bf16_t *g, hipStream_t s) {
    if (count <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid), dim3(256), 0, s, dy, y, count, g);
    return hip_fail(hipGetLastError(), "k_relu_bwd");
}

// one thread per (output pixel, 8 channels)
__global__ void k_pool2_fwd(const bf16_t *x, int c, int n, int h, int w, bf16_t *y, uint8_t *idx) {
    const int ho = h / 2, wo = w / 2, cg = c / 8;
    const int64_t total = (int64_t)n * ho * wo * cg;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int g8 = (int)(t % cg);
        const int64_t q = t / cg;
        const int j = (int)(q % wo);
        const int64_t q2 = q / wo;
        const int i = (int)(q2 % ho);
        const int im = (int)(q2 / ho);
        V8 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t sp = ((int64_t)im * h + 2 * i + (k >> 1)) * w + 2 * j + (k & 1);
            v[k].u = *reinterpret_cast<const uint4 *>(x + sp * c + g8 * 8);
        }
        V8 o;
        uint8_t id[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float best = bf2f(v[0].h[e]);
            int bi = 0;
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                const float f = bf2f(v[k].h[e]);
                if (f > best) {
                    best = f;
                    bi = k;
                }
            }
            o.h[e] = v[bi].h[e];
            id[e] = (uint8_t)bi;
        }
        *reinterpret_cast<uint4 *>(y + q * c + g8 * 8) = o.u;
#pragma unroll
        for (int e = 0; e < 8; ++e) idx[q * c + g8 * 8 + e] = id[e];
    }
}

int nn_pool2_fwd(const bf16_t *x, int c, int n, int h, int w, bf16_t *y, uint8_t *idx, hipStream_t s) {
    if (c % 8 || h % 2 || w % 2) {
        set_error("nn pool2: channels must be a multiple of 8 and the size even");
        return RT_EINVAL;
    }
    const int64_t total = (int64_t)n * (h / 2) * (w / 2) * (c / 8);
    if (total <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_pool2_fwd, dim3(grid), dim3(256), 0, s, x, c, n, h, w, y, idx);
    return hip_fail(hipGetLastError(), "k_pool2_fwd");
}

// one thread per (output pixel, channel); windows are disjoint
__global__ void k_pool2_bwd(const float *dy, const uint8_t *idx, int c, int n, int h, int w, float *dx) {
    const int ho = h / 2, wo = w / 2;
    const int64_t total = (int64_t)n * ho * wo * c;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int ch = (int)(t % c);
        const int64_t q = t / c;
        const int j = (int)(q % wo);
        const int64_t q2 = q / wo;
        const int i = (int)(q2 % ho);
        const int im = (int)(q2 / ho);
        const int k = idx[t];
        const int64_t sp = ((int64_t)im * h + 2 * i + (k >> 1)) * w + 2 * j + (k & 1);
        dx[sp * c + ch] += dy[t];
    }
}

int nn_pool2_bwd(const float *dy, const uint8_t *idx, int c, int n, int h, int w, float *dx, hipStream_t s) {
    const int64_t total = (int64_t)n * (h / 2) * (w / 2) * c;
    if (total <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid), dim3(256), 0, s, dy, idx, c, n, h, w, dx);
    return hip_fail(hipGetLastError(), "k_pool2_bwd");
}

__global__ void k_prep_input(const uint8_t *rgb, int64_t pitch, int iw, int ih, const int32_t *ox, const int32_t *oy,
                             int n, int h, int w, bf16_t *x) {
    const int64_t total = (int64_t)n * h * w;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(p / ((int64_t)h * w));
        const int rem = (int)(p - (int64_t)k * h * w);
        const int y = rem / w, xx = rem - (rem / w) * w;
        const int sy = oy[k] + y, sx = ox[k] + xx;
        V8 o;
        o.u = make_uint4(0, 0, 0, 0);
        if (sy >= 0 && sy < ih && sx >= 0 && sx < iw) {
            const uint8_t *px = rgb + (int64_t)sy * pitch + 3 * (int64_t)sx;
#pragma unroll
            // v / 255 - 0.5 = (2v - 255) / 510: an exact numerator and one
            // correctly rounded division
            for (int c = 0; c < 3; ++c) o.h[c] = f2bf((float)(2 * (int)px[c] - 255) / 510.0f);
        }
        *reinterpret_cast<uint4 *>(x + p * 8) = o.u;
    }
}

int nn_prep_input(const uint8_t *rgb, int64_t pitch, int iw, int ih, const int32_t *ox, const int32_t *oy, int n,
                  int h, int w, bf16_t *x, hipStream_t s) {
    const int64_t total = (int64_t)n * h * w;
    if (total <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_prep_input, dim3(grid), dim3(256), 0, s, rgb, pitch, iw, ih, ox, oy, n, h, w, x);
    return hip_fail(hipGetLastError(), "k_prep_input");
}

// one thread per pixel; block sums of the loss and of the head gradients
__global__ __launch_bounds__(256) void k_head(HeadArgs a) {
    __shared__ float red[35][8];
    const int64_t P = (int64_t)a.n * a.h * a.w;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool on = p < P;
    float x[16];
    V8 v0, v1;
    if (on) {
        v0.u = *reinterpret_cast<const uint4 *>(a.x + p * 16);
        v1.u = *reinterpret_cast<const uint4 *>(a.x + p * 16 + 8);
    } else {
        v0.u = v1.u = make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = bf2f(v0.h[c]);
        x[c + 8] = bf2f(v1.h[c]);
    }
    float z[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 16; ++c) s += a.wh[o * 16 + c] * x[c];
        z[o] = s + a.bh[o];
    }
    if (!a.t_fg) {   // inference: probabilities into the kept part of the window
        if (!on) return;
        const int64_t hw = (int64_t)a.h * a.w;
        const int k = (int)(p / hw);
        const int rem = (int)(p - k * hw);
        const int y = rem / a.w, xx = rem - (rem / a.w) * a.w;
        const int32_t *kp = a.keep + 4 * k;
        if (xx < kp[0] || xx >= kp[1] || y < kp[2] || y >= kp[3]) return;
        const int oy = a.oy[k] + y, ox = a.ox[k] + xx;
        if (oy < 0 || oy >= a.out_h || ox < 0 || ox >= a.out_w) return;
        a.p_fg[(int64_t)oy * a.pitch + ox] = 1.f / (1.f + expf(-z[0]));
        a.p_seed[(int64_t)oy * a.pitch + ox] = 1.f / (1.f + expf(-z[1]));
        return;
    }
    const float inv = 1.f / (float)P;
    float part[35];
#pragma unroll
    for (int k = 0; k < 35; ++k) part[k] = 0.f;
    if (on) {
        const float t[2] = {(float)a.t_fg[p], (float)a.t_seed[p]};
        const float wgt[2] = {1.f, a.w_seed};
        float gz[2], lsum = 0.f;
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const float zz = z[o];
            lsum += wgt[o] * ((zz > 0.f ? zz : 0.f) - zz * t[o] + log1pf(expf(-fabsf(zz))));
            gz[o] = wgt[o] * (1.f / (1.f + expf(-zz)) - t[o]) * inv;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) a.dx[p * 16 + c] = a.wh[c] * gz[0] + a.wh[16 + c] * gz[1];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
#pragma unroll
            for (int c = 0; c < 16; ++c) part[o * 16 + c] = gz[o] * x[c];
            part[32 + o] = gz[o];
        }
        part[34] = lsum * inv;
    }
    // wave reduction, then one partial per wave in LDS
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 35; ++k) {
        float v = part[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 35) {
        float s = 0.f;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) s += red[threadIdx.x][wv];
        if (threadIdx.x < 32)
            atomicAdd(a.dw + threadIdx.x, s);
        else if (threadIdx.x < 34)
            atomicAdd(a.db + threadIdx.x - 32, s);
        else
            atomicAdd(a.loss, s);
    }
}

int nn_head(const HeadArgs &a, hipStream_t s) {
    const int64_t P = (int64_t)a.n * a.h * a.w;
    if (P <= 0) return RT_OK;
    hipLaunchKernelGGL(k_head, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, a);
    return hip_fail(hipGetLastError(), "k_head");
}

__global__ void k_adam(float *p, float *g, float *m, float *v, int64_t count, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        g[i] = 0.f;
    }
}

int nn_adam(float *p, float *g, float *m, float *v, int64_t count, float lr, float b1, float b2, float eps, int t,
            hipStream_t s) {
    if (count <= 0) return RT_OK;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
    const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adam, dim3(grid), dim3(256), 0, s, p, g, m, v, count, lr, b1, b2, eps, c1, c2);
    return hip_fail(hipGetLastError(), "k_adam");
}

__global__ void k_pack_conv3(const float *w, int co, int ci, bf16_t *wf, bf16_t *wt) {
    const int64_t total = (int64_t)co * 9 * ci;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % ci);
        const int tap = (int)((i / ci) % 9);
        const int o = (int)(i / (9 * (int64_t)ci));
        const bf16_t b = f2bf(w[i]);
        wf[i] = b;
        if (wt) wt[((int64_t)c * 9 + tap) * co + o] = b;
    }
}

int nn_pack_conv3(const float *w, int co, int ci, bf16_t *wf, bf16_t *wt, hipStream_t s) {
    const int64_t total = (int64_t)co * 9 * ci;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_conv3, dim3(grid), dim3(256), 0, s, w, co, ci, wf, wt);
    return hip_fail(hipGetLastError(), "k_pack_conv3");
}

__global__ void k_pack_up2(const float *w, int ci, int co, bf16_t *uf, bf16_t *ut) {
    const int64_t total = (int64_t)ci * 4 * co;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int o = (int)(i % co);
        const int ab = (int)((i / co) % 4);
        const int c = (int)(i / (4 * (int64_t)co));
        const bf16_t b = f2bf(w[i]);
        ut[i] = b;
        uf[((int64_t)ab * co + o) * ci + c] = b;
    }
}

int nn_pack_up2(const float *w, int ci, int co, bf16_t *uf, bf16_t *ut, hipStream_t s) {
    const int64_t total = (int64_t)ci * 4 * co;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_up2, dim3(grid), dim3(256), 0, s, w, ci, co, uf, ut);
    return hip_fail(hipGetLastError(), "k_pack_up2");
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

int nn_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return RT_OK;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid), dim3(256), 0, s, p, v, n);
    return hip_fail(hipGetLastError(), "k_fill_f32");
}

}  // namespace rtseg
