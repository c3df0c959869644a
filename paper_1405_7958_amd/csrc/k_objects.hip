// Pre-Watershed + Watershed, one workgroup per connected component.
//
// The paper restructures feature computation into one bounding box per
// nucleus, one GPU block per box (Sec. 5.1); the same decomposition serves
// the watershed stage here.  Everything after the area filter (distance
// transform, h-maxima seeds, flood, cut, relabelling, final area filter)
// depends only on the component itself:
//   * the nearest background pixel of a component pixel lies in the
//     component's bounding box grown by one pixel (the open disc of radius d
//     around p holds no background pixel, so it is a connected foreground set
//     and belongs to the component; the background pixel that ends the disc
//     is 8-adjacent to the component), so the distance transform computed in
//     that crop with "not in the component" as background is exact;
//   * the reconstructions run on the graph of the component's pixels, and
//     components are not 8-adjacent to each other.
// The crop state (flags, Dq, two work planes and the flood keys) lives in LDS
// when it fits; larger crops run the same code on a global scratch slice.
#include "rt_internal.h"

#include <climits>

namespace rtseg {

constexpr int OBJ_THREADS = 256;
constexpr int LDS_CAP = 3072;  // crop pixels held in LDS
constexpr int NEGV = INT_MIN;
constexpr int GINF = 1 << 28;

enum : uint8_t { F_IN = 1, F_RM = 2, F_M = 4 };

template <typename KeyT>
struct KeyTraits;
template <>
struct KeyTraits<uint32_t> {  // crop < 4096 pixels: dist and label fit in 12 bits each
    static constexpr int SH = 12;
    static constexpr uint32_t INF = 0xffffffffu;
};
template <>
struct KeyTraits<uint64_t> {
    static constexpr int SH = 32;
    static constexpr uint64_t INF = ~0ull;
};

template <typename KeyT>
struct Crop {
    uint8_t *fl;
    int32_t *dq;
    int32_t *A;
    int32_t *B;
    KeyT *K;
};

struct Shape {
    int cx0, cy0, cw, ch, n;
};

__device__ __forceinline__ int isqrt_exact(int64_t v) {
    if (v <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (int)r;
}

// union-find on a crop plane (LDS or global); roots are the smallest index
__device__ __forceinline__ int cfind(int32_t *P, int x) {
    int p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        x = p;
        p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return x;
}
__device__ __forceinline__ void cunite(int32_t *P, int a, int b) {
    for (;;) {
        a = cfind(P, a);
        b = cfind(P, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        int old = atomicMin(P + a, b);
        if (old == a) return;
        a = old;
    }
}

// Labels the pixels whose flag bit `bit` is set by 8-connected components:
// P[i] = smallest crop index of the component, -1 elsewhere.
__device__ void crop_ccl(const Shape &s, const uint8_t *fl, uint8_t bit, int32_t *P) {
    for (int i = threadIdx.x; i < s.n; i += blockDim.x) P[i] = (fl[i] & bit) ? i : -1;
    __syncthreads();
    for (int i = threadIdx.x; i < s.n; i += blockDim.x) {
        if (!(fl[i] & bit)) continue;
        int c = i % s.cw, r = i / s.cw;
        if (c > 0 && (fl[i - 1] & bit)) cunite(P, i, i - 1);
        if (r > 0) {
            if (fl[i - s.cw] & bit) cunite(P, i, i - s.cw);
            if (c > 0 && (fl[i - s.cw - 1] & bit)) cunite(P, i, i - s.cw - 1);
            if (c < s.cw - 1 && (fl[i - s.cw + 1] & bit)) cunite(P, i, i - s.cw + 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s.n; i += blockDim.x)
        if (fl[i] & bit) P[i] = cfind(P, i);
    __syncthreads();
}

// V <- reconstruction of V under M on the graph of in-component pixels
// (8-connected), by in-place relaxation until nothing changes.
__device__ void crop_recon(const Shape &s, const uint8_t *fl, int32_t *V, const int32_t *M) {
    for (int it = 0;; ++it) {
        bool ch = false;
        const bool fwd = (it & 1) == 0;
        for (int k = threadIdx.x; k < s.n; k += blockDim.x) {
            int i = fwd ? k : s.n - 1 - k;
            if (!(fl[i] & F_IN)) continue;
            int c = i % s.cw, r = i / s.cw;
            int m = NEGV;
            for (int dy = -1; dy <= 1; ++dy) {
                int rr = r + dy;
                if (rr < 0 || rr >= s.ch) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    int cc = c + dx;
                    if ((dx | dy) == 0 || cc < 0 || cc >= s.cw) continue;
                    int j = rr * s.cw + cc;
                    if (fl[j] & F_IN) m = max(m, V[j]);
                }
            }
            int nv = min(m, M[i]);
            if (nv > V[i]) {
                V[i] = nv;
                ch = true;
            }
        }
        if (!__syncthreads_or(ch)) break;
    }
}

__device__ int block_max(int v, int *red) {
    if (threadIdx.x == 0) *red = NEGV;
    __syncthreads();
    if (v != NEGV) atomicMax(red, v);
    __syncthreads();
    int r = *red;
    __syncthreads();
    return r;
}

template <typename KeyT>
__device__ void process_object(const ObjArgs &a, int g, const Shape &s, Crop<KeyT> m, int *red) {
    using KT = KeyTraits<KeyT>;
    const int n = s.n;
    // ---- load the component's pixels
    bool zero = false;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int px = s.cx0 + i % s.cw, py = s.cy0 + i / s.cw;
        bool in = a.labels[(int64_t)py * a.pitch + px] == g;
        m.fl[i] = in ? F_IN : 0;
        zero |= !in;
    }
    const bool has_zero = __syncthreads_or(zero) && a.tile_has_zero;

    // ---- exact distance transform inside the crop
    for (int c = threadIdx.x; c < s.cw; c += blockDim.x) {
        int run = GINF;
        for (int r = 0; r < s.ch; ++r) {
            int i = r * s.cw + c;
            run = (m.fl[i] & F_IN) ? (run < GINF ? run + 1 : GINF) : 0;
            m.A[i] = run;
        }
        run = GINF;
        for (int r = s.ch - 1; r >= 0; --r) {
            int i = r * s.cw + c;
            run = (m.fl[i] & F_IN) ? (run < GINF ? run + 1 : GINF) : 0;
            if (run < m.A[i]) m.A[i] = run;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!(m.fl[i] & F_IN)) {
            m.dq[i] = 0;
            continue;
        }
        if (!has_zero) {
            m.dq[i] = RT_DQ_MAX;
            continue;
        }
        int c = i % s.cw, r = i / s.cw;
        const int32_t *row = m.A + r * s.cw;
        int64_t best = row[c] < GINF ? (int64_t)row[c] * row[c] : INT64_MAX;
        for (int dx = 1;; ++dx) {
            int64_t dd = (int64_t)dx * dx;
            if (dd >= best) break;
            bool lo = c - dx >= 0, hi = c + dx < s.cw;
            if (!lo && !hi) break;
            if (lo && row[c - dx] < GINF) best = min(best, dd + (int64_t)row[c - dx] * row[c - dx]);
            if (hi && row[c + dx] < GINF) best = min(best, dd + (int64_t)row[c + dx] * row[c + dx]);
        }
        m.dq[i] = isqrt_exact(4 * best);
    }
    __syncthreads();

    // ---- seeds
    if (a.seeds) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int px = s.cx0 + i % s.cw, py = s.cy0 + i / s.cw;
            if ((m.fl[i] & F_IN) && a.seeds[(int64_t)py * a.pitch + px]) m.fl[i] |= F_RM;
        }
        __syncthreads();
    } else {
        // g = recon(Dq - h under Dq)
        for (int i = threadIdx.x; i < n; i += blockDim.x) m.A[i] = (m.fl[i] & F_IN) ? m.dq[i] - a.h_seed : NEGV;
        __syncthreads();
        crop_recon(s, m.fl, m.A, m.dq);
        // regional maxima: g - recon(g - 1 under g) > 0
        for (int i = threadIdx.x; i < n; i += blockDim.x) m.B[i] = (m.fl[i] & F_IN) ? m.A[i] - 1 : NEGV;
        __syncthreads();
        crop_recon(s, m.fl, m.B, m.A);
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.A[i] - m.B[i] > 0) m.fl[i] |= F_RM;
        __syncthreads();
    }
    crop_ccl(s, m.fl, F_RM, m.B);  // B = seed label (crop index of the seed component root) or -1

    // ---- lambda = recon(Dq on seeds under Dq)
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        m.A[i] = ((m.fl[i] & F_IN) && (m.fl[i] & F_RM)) ? m.dq[i] : NEGV;
    __syncthreads();
    crop_recon(s, m.fl, m.A, m.dq);

    // ---- flood, level by level from the highest lambda
    for (;;) {
        int lv = NEGV;
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] != NEGV) lv = max(lv, m.A[i]);
        const int L = block_max(lv, red);
        if (L == NEGV) break;
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] == L) m.K[i] = KT::INF;
        __syncthreads();
        for (int it = 0;; ++it) {
            bool ch = false;
            const bool fwd = (it & 1) == 0;
            for (int k = threadIdx.x; k < n; k += blockDim.x) {
                int i = fwd ? k : n - 1 - k;
                if (!((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] == L)) continue;
                int c = i % s.cw, r = i / s.cw;
                KeyT best = m.K[i];
                for (int dy = -1; dy <= 1; ++dy) {
                    int rr = r + dy;
                    if (rr < 0 || rr >= s.ch) continue;
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cc = c + dx;
                        if ((dx | dy) == 0 || cc < 0 || cc >= s.cw) continue;
                        int j = rr * s.cw + cc;
                        if (!(m.fl[j] & F_IN)) continue;
                        KeyT cand = KT::INF;
                        if (m.B[j] >= 0)
                            cand = ((KeyT)1 << KT::SH) | (KeyT)m.B[j];
                        else if (m.A[j] == L && m.K[j] != KT::INF)
                            cand = m.K[j] + ((KeyT)1 << KT::SH);
                        if (cand < best) best = cand;
                    }
                }
                if (best < m.K[i]) {
                    m.K[i] = best;
                    ch = true;
                }
            }
            if (!__syncthreads_or(ch)) break;
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] == L)
                m.B[i] = (int32_t)(m.K[i] & (((KeyT)1 << KT::SH) - 1));
        __syncthreads();
    }
    // ---- leftovers (external seeds only): their own components
    if (a.seeds) {
        bool left = false;
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.B[i] < 0) {
                m.fl[i] |= F_M;  // temporary use of the M bit
                left = true;
            }
        if (__syncthreads_or(left)) {
            crop_ccl(s, m.fl, F_M, m.A);
            for (int i = threadIdx.x; i < n; i += blockDim.x)
                if (m.fl[i] & F_M) m.B[i] = m.A[i];
            __syncthreads();
        }
        for (int i = threadIdx.x; i < n; i += blockDim.x) m.fl[i] &= (uint8_t)~F_M;
        __syncthreads();
    }

    // ---- cut: keep p iff no neighbour in the component has a smaller label
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!(m.fl[i] & F_IN)) continue;
        int c = i % s.cw, r = i / s.cw;
        int lab = m.B[i];
        bool keep = true;
        for (int dy = -1; dy <= 1 && keep; ++dy) {
            int rr = r + dy;
            if (rr < 0 || rr >= s.ch) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int cc = c + dx;
                if ((dx | dy) == 0 || cc < 0 || cc >= s.cw) continue;
                int j = rr * s.cw + cc;
                if ((m.fl[j] & F_IN) && m.B[j] < lab) {
                    keep = false;
                    break;
                }
            }
        }
        if (keep) m.fl[i] |= F_M;
    }
    __syncthreads();
    // ---- relabel the kept pixels, count areas
    crop_ccl(s, m.fl, F_M, m.A);
    for (int i = threadIdx.x; i < n; i += blockDim.x) m.dq[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (m.fl[i] & F_M) atomicAdd(m.dq + m.A[i], 1);
    __syncthreads();
    int kept = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!(m.fl[i] & F_IN)) continue;
        int px = s.cx0 + i % s.cw, py = s.cy0 + i / s.cw;
        int64_t o = (int64_t)py * a.pitch + px;
        int lab = 0;
        if (m.fl[i] & F_M) {
            int root = m.A[i];
            int ar = m.dq[root];
            bool ok = ar >= a.min_area && (a.max_area < 0 || ar <= a.max_area);
            if (ok) {
                lab = (s.cy0 + root / s.cw) * a.w + s.cx0 + root % s.cw + 1;
                if (root == i) ++kept;
            }
        }
        a.labels[o] = lab;
        a.mask[o] = lab ? 1 : 0;
    }
    if (a.n_kept && kept) atomicAdd(a.n_kept, kept);
    __syncthreads();
}

__device__ bool object_shape(const ObjArgs &a, int g, Shape &s) {
    s.cx0 = max(0, a.st_x0[g] - 1);
    s.cy0 = max(0, a.st_y0[g] - 1);
    int cx1 = min(a.w - 1, a.st_x1[g] + 1), cy1 = min(a.h - 1, a.st_y1[g] + 1);
    s.cw = cx1 - s.cx0 + 1;
    s.ch = cy1 - s.cy0 + 1;
    s.n = s.cw * s.ch;
    return true;
}

__device__ void erase_object(const ObjArgs &a, int g, const Shape &s) {
    for (int i = threadIdx.x; i < s.n; i += blockDim.x) {
        int px = s.cx0 + i % s.cw, py = s.cy0 + i / s.cw;
        int64_t o = (int64_t)py * a.pitch + px;
        if (a.labels[o] == g) {
            a.labels[o] = 0;
            a.mask[o] = 0;
        }
    }
}

__global__ __launch_bounds__(OBJ_THREADS) void k_objects(ObjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int red;
    Crop<uint32_t> m;
    m.dq = (int32_t *)smem;
    m.A = m.dq + LDS_CAP;
    m.B = m.A + LDS_CAP;
    m.K = (uint32_t *)(m.B + LDS_CAP);
    m.fl = (uint8_t *)(m.K + LDS_CAP);
    const int nobj = *a.n_obj;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int g = a.obj_list[o];
        Shape s;
        object_shape(a, g, s);
        if (a.st_area[g] < a.min_area_pre) {
            erase_object(a, g, s);
            continue;
        }
        if (s.n > LDS_CAP) {
            if (threadIdx.x == 0) a.big_list[atomicAdd(a.n_big, 1)] = g;
            continue;
        }
        process_object<uint32_t>(a, g, s, m, &red);
    }
}

__global__ __launch_bounds__(OBJ_THREADS) void k_objects_big(ObjArgs a, size_t per_block) {
    __shared__ int red;
    const int nbig = *a.n_big;
    char *base = (char *)a.big_scratch + per_block * blockIdx.x;
    for (int o = blockIdx.x; o < nbig; o += gridDim.x) {
        const int g = a.big_list[o];
        Shape s;
        object_shape(a, g, s);
        Crop<uint64_t> m;
        m.K = (uint64_t *)base;
        m.dq = (int32_t *)(m.K + s.n);
        m.A = m.dq + s.n;
        m.B = m.A + s.n;
        m.fl = (uint8_t *)(m.B + s.n);
        process_object<uint64_t>(a, g, s, m, &red);
    }
}

int launch_objects(const ObjArgs &a, hipStream_t s) {
    size_t lds = (size_t)LDS_CAP * (4 * 4 + 1);
    int grid = a.max_obj;
    hipLaunchKernelGGL(k_objects, dim3(grid), dim3(OBJ_THREADS), lds, s, a);
    return hip_fail(hipGetLastError(), "k_objects");
}

// bytes of global scratch one big object of `n` crop pixels needs
size_t big_object_bytes(size_t n) { return n * (8 + 4 * 3 + 1) + 256; }

int launch_objects_big(const ObjArgs &a, int n_big_host, hipStream_t s) {
    if (n_big_host <= 0) return RT_OK;
    size_t per = big_object_bytes((size_t)a.w * a.h);
    per = (per + 255) & ~size_t(255);
    size_t cap_blocks = a.big_scratch_elems * sizeof(int32_t) / per;
    int grid = (int)std::min<size_t>((size_t)n_big_host, cap_blocks);
    if (grid < 1) {
        set_error("objects: big-object scratch too small");
        return RT_ENOMEM;
    }
    hipLaunchKernelGGL(k_objects_big, dim3(grid), dim3(OBJ_THREADS), 0, s, a, per);
    return hip_fail(hipGetLastError(), "k_objects_big");
}

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

__global__ void k_count_zero(const uint8_t *m, int w, int h, int64_t pitch, int32_t *out) {
    int64_t n = (int64_t)w * h;
    int c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        c += m[y * pitch + x] == 0;
    }
    if (__syncthreads_or(c > 0) && threadIdx.x == 0) atomicAdd(out, 1);
}
int launch_count_zero(const uint8_t *m, int w, int h, int64_t pitch, int32_t *out, hipStream_t s) {
    int64_t n = (int64_t)w * h;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_count_zero, dim3(grid), dim3(256), 0, s, m, w, h, pitch, out);
    return hip_fail(hipGetLastError(), "k_count_zero");
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
