// Connected-component labelling by union-find (BWLabel, Sec. 5.1: a forest
// in which every pixel starts as its own tree, adjacent trees are merged, and
// labels are read off by flattening the trees).
//
// Three launches over 32 x 32 tiles (one 256-thread workgroup per tile):
//   local : the tile's predicate is staged in LDS and a union-find forest is
//           built there with LDS atomicMin (a root is always the smallest
//           index of its tree, so labels are canonical by construction).
//           Only the tile's roots and its edge pixels are published to the
//           global id array (id 0 = virtual node, pixel p = id p + 1).
//   merge : one thread per pair of pixels facing each other across a tile
//           edge unites their global trees with atomicMin.
//   flatten: the tile's forest is rebuilt in LDS (1 byte/pixel of input
//           instead of storing 4 bytes/pixel of local roots), each local root
//           finds its global root once, and the per-pixel result is written.
//
// The same engine serves FillHoles (background components joined to a virtual
// frame node), BWLabel with per-component area and bounding box, and the
// multi-level frame-connectivity lower bound used to start the grayscale
// reconstruction.
#include "rt_internal.h"

namespace rtseg {

constexpr int TW = 32, TH = 32, TN = TW * TH, NT = 256;
constexpr int MAXLEV = 8;

__device__ __forceinline__ int ld_agent(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lfind(volatile int *P, int x) {
    int p = P[x];
    while (p != x) {
        x = p;
        p = P[x];
    }
    return x;
}

__device__ __forceinline__ void lunite(int *P, int a, int b) {
    for (;;) {
        a = lfind(P, a);
        b = lfind(P, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        int old = atomicMin(&P[a], b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ int gfind(int32_t *ids, int x) {
    int p = ld_agent(ids + x);
    while (p != x) {
        x = p;
        p = ld_agent(ids + x);
    }
    return x;
}

__device__ __forceinline__ void gunite(int32_t *ids, int a, int b) {
    for (;;) {
        a = gfind(ids, a);
        b = gfind(ids, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        int old = atomicMin(ids + a, b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ bool eval_pred(const CclArgs &A, int x, int y, int level) {
    switch (A.pred) {
        case CclPred::NonZero: return A.a[(int64_t)y * A.pitch_a + x] != 0;
        case CclPred::Zero: return A.a[(int64_t)y * A.pitch_a + x] == 0;
        case CclPred::TophatBg:
            return (int)A.a[(int64_t)y * A.pitch_a + x] - (int)A.b[(int64_t)y * A.pitch_b + x] < A.t;
        case CclPred::Level: return (int)A.a[(int64_t)y * A.pitch_a + x] >= level;
    }
    return false;
}

struct TileCtx {
    int x0, y0, tw, th;
};

// Builds the LDS forest of the tile for predicate bits `pr` (1 = member).
// Non-members get P = -1.  Ends with P[i] = local root for every member.
__device__ void tile_forest(const uint8_t *pr, int *P, int conn, const TileCtx &tc) {
    for (int i = threadIdx.x; i < TN; i += NT) P[i] = pr[i] ? i : -1;
    __syncthreads();
    for (int i = threadIdx.x; i < TN; i += NT) {
        if (!pr[i]) continue;
        int lx = i % TW, ly = i / TW;
        if (lx > 0 && pr[i - 1]) lunite(P, i, i - 1);
        if (ly > 0) {
            if (pr[i - TW]) lunite(P, i, i - TW);
            if (conn == 8) {
                if (lx > 0 && pr[i - TW - 1]) lunite(P, i, i - TW - 1);
                if (lx < TW - 1 && pr[i - TW + 1]) lunite(P, i, i - TW + 1);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TN; i += NT)
        if (pr[i]) P[i] = lfind(P, i);
    __syncthreads();
}

__device__ __forceinline__ int pix_id(const CclArgs &A, const TileCtx &tc, int i) {
    return (tc.y0 + i / TW) * A.w + tc.x0 + i % TW + 1;
}

// Stages the predicate (or, for Level, the Hq tile) into LDS.  Pixels beyond
// the image edge are non-members.
__device__ void stage_tile(const CclArgs &A, const TileCtx &tc, uint8_t *raw) {
    for (int i = threadIdx.x; i < TN; i += NT) {
        int lx = i % TW, ly = i / TW;
        uint8_t v = 0;
        if (lx < tc.tw && ly < tc.th) {
            int x = tc.x0 + lx, y = tc.y0 + ly;
            if (A.pred == CclPred::Level)
                v = A.a[(int64_t)y * A.pitch_a + x];
            else
                v = eval_pred(A, x, y, 0) ? 1 : 0;
        }
        raw[i] = v;
    }
    __syncthreads();
}

__device__ void level_bits(const uint8_t *raw, uint8_t *pr, int level, const TileCtx &tc) {
    for (int i = threadIdx.x; i < TN; i += NT) {
        int lx = i % TW, ly = i / TW;
        pr[i] = (lx < tc.tw && ly < tc.th && (int)raw[i] >= level) ? 1 : 0;
    }
    __syncthreads();
}

__device__ __forceinline__ bool on_frame(const CclArgs &A, int x, int y) {
    return x == 0 || y == 0 || x == A.w - 1 || y == A.h - 1;
}

// --------------------------------------------------------------------------
// local phase
// --------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_ccl_local(CclArgs A) {
    __shared__ uint8_t raw[TN];
    __shared__ uint8_t pr[TN];
    __shared__ uint8_t fr[TN];
    __shared__ int P[TN];
    const int ntx = (A.w + TW - 1) / TW;
    TileCtx tc;
    tc.x0 = (blockIdx.x % ntx) * TW;
    tc.y0 = (blockIdx.x / ntx) * TH;
    tc.tw = min(TW, A.w - tc.x0);
    tc.th = min(TH, A.h - tc.y0);
    stage_tile(A, tc, raw);
    const int nlev = A.pred == CclPred::Level ? A.n_levels : 1;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    for (int lev = 0; lev < nlev; ++lev) {
        const uint8_t *bits = raw;
        if (A.pred == CclPred::Level) {
            level_bits(raw, pr, A.levels[lev], tc);
            bits = pr;
        }
        tile_forest(bits, P, A.conn, tc);
        int32_t *ids = A.ids + lev * nid;
        for (int i = threadIdx.x; i < TN; i += NT) fr[i] = 0;
        __syncthreads();
        if (A.frame_virtual) {
            for (int i = threadIdx.x; i < TN; i += NT) {
                if (!bits[i]) continue;
                if (on_frame(A, tc.x0 + i % TW, tc.y0 + i / TW)) fr[P[i]] = 1;
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < TN; i += NT) {
            if (!bits[i]) continue;
            int lx = i % TW, ly = i / TW;
            int r = P[i];
            int id = pix_id(A, tc, i);
            if (r == i) {
                ids[id] = fr[i] ? 0 : id;
                if (A.st_area) {
                    A.st_area[id] = 0;
                    A.st_x0[id] = 0x7fffffff;
                    A.st_y0[id] = 0x7fffffff;
                    A.st_x1[id] = -1;
                    A.st_y1[id] = -1;
                }
            } else if (lx == 0 || ly == 0 || lx == tc.tw - 1 || ly == tc.th - 1) {
                ids[id] = pix_id(A, tc, r);
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// merge phase: pairs across tile edges
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ccl_merge(CclArgs A, int64_t n_vert) {
    const int ntx = (A.w + TW - 1) / TW, nty = (A.h + TH - 1) / TH;
    int64_t n_hor = (int64_t)(nty - 1) * A.w;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_vert + n_hor) return;
    const int nlev = A.pred == CclPred::Level ? A.n_levels : 1;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    int px, py, qx[3], qy[3], nq = 0;
    if (t < n_vert) {
        int bx = (int)(t / A.h) + 1;
        py = (int)(t % A.h);
        px = bx * TW - 1;
        if (A.conn == 8) {
            for (int d = -1; d <= 1; ++d)
                if (py + d >= 0 && py + d < A.h) { qx[nq] = px + 1; qy[nq] = py + d; ++nq; }
        } else {
            qx[0] = px + 1; qy[0] = py; nq = 1;
        }
    } else {
        int64_t u = t - n_vert;
        int by = (int)(u / A.w) + 1;
        px = (int)(u % A.w);
        py = by * TH - 1;
        if (A.conn == 8) {
            for (int d = -1; d <= 1; ++d)
                if (px + d >= 0 && px + d < A.w) { qx[nq] = px + d; qy[nq] = py + 1; ++nq; }
        } else {
            qx[0] = px; qy[0] = py + 1; nq = 1;
        }
    }
    (void)ntx;
    for (int lev = 0; lev < nlev; ++lev) {
        int level = A.pred == CclPred::Level ? A.levels[lev] : 0;
        if (!eval_pred(A, px, py, level)) continue;
        int32_t *ids = A.ids + lev * nid;
        int pid = py * A.w + px + 1;
        for (int k = 0; k < nq; ++k)
            if (eval_pred(A, qx[k], qy[k], level)) gunite(ids, pid, qy[k] * A.w + qx[k] + 1);
    }
}

// --------------------------------------------------------------------------
// flatten phase + outputs
// --------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_ccl_flatten(CclArgs A) {
    __shared__ uint8_t raw[TN];
    __shared__ uint8_t pr[TN];
    __shared__ uint8_t best[TN];
    __shared__ int P[TN];
    __shared__ int G[TN];
    __shared__ int cnt[TN];
    __shared__ uint32_t cmask[TN];
    __shared__ uint32_t rmask[TN];
    const int ntx = (A.w + TW - 1) / TW;
    TileCtx tc;
    tc.x0 = (blockIdx.x % ntx) * TW;
    tc.y0 = (blockIdx.x / ntx) * TH;
    tc.tw = min(TW, A.w - tc.x0);
    tc.th = min(TH, A.h - tc.y0);
    stage_tile(A, tc, raw);
    const int64_t nid = (int64_t)A.w * A.h + 1;

    if (A.out == CclOut::LevelBound) {
        for (int i = threadIdx.x; i < TN; i += NT) best[i] = 0;
        __syncthreads();
        for (int lev = 0; lev < A.n_levels; ++lev) {
            int level = A.levels[lev];
            level_bits(raw, pr, level, tc);
            tile_forest(pr, P, A.conn, tc);
            int32_t *ids = A.ids + lev * nid;
            for (int i = threadIdx.x; i < TN; i += NT)
                if (pr[i] && P[i] == i) G[i] = gfind(ids, pix_id(A, tc, i));
            __syncthreads();
            for (int i = threadIdx.x; i < TN; i += NT)
                if (pr[i] && G[P[i]] == 0 && level > best[i]) best[i] = (uint8_t)level;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < TN; i += NT) {
            int lx = i % TW, ly = i / TW;
            if (lx >= tc.tw || ly >= tc.th) continue;
            int x = tc.x0 + lx, y = tc.y0 + ly;
            int j = on_frame(A, x, y) ? raw[i] : 0;
            int v = best[i] > j ? best[i] : j;
            A.bound[(int64_t)y * A.pitch_r + x] = (uint8_t)v;
        }
        return;
    }

    tile_forest(raw, P, A.conn, tc);
    for (int i = threadIdx.x; i < TN; i += NT) {
        if (raw[i] && P[i] == i) G[i] = gfind(A.ids, pix_id(A, tc, i));
        cnt[i] = 0;
        cmask[i] = 0;
        rmask[i] = 0;
    }
    __syncthreads();
    const bool stats = A.out == CclOut::Labels && A.st_area != nullptr;
    for (int i = threadIdx.x; i < TN; i += NT) {
        int lx = i % TW, ly = i / TW;
        if (lx >= tc.tw || ly >= tc.th) continue;
        int x = tc.x0 + lx, y = tc.y0 + ly;
        if (A.out == CclOut::Labels) {
            int lab = raw[i] ? G[P[i]] : 0;
            A.labels[(int64_t)y * A.pitch_l + x] = lab;
            if (!raw[i] && A.bg_zero_mask) A.bg_zero_mask[(int64_t)y * A.pitch_m + x] = 0;
            if (stats && raw[i]) {
                int r = P[i];
                atomicAdd(&cnt[r], 1);
                atomicOr(&cmask[r], 1u << lx);
                atomicOr(&rmask[r], 1u << ly);
            }
        } else {  // FillHoles: members are background pixels of F0
            uint8_t f = raw[i] ? (G[P[i]] != 0 ? 1 : 0) : 1;
            A.fill[(int64_t)y * A.pitch_f + x] = f;
        }
    }
    if (!stats && !(A.out == CclOut::Labels && A.obj_list)) return;
    __syncthreads();
    for (int i = threadIdx.x; i < TN; i += NT) {
        if (!raw[i] || P[i] != i) continue;
        int g = G[i];
        if (stats) {
            atomicAdd(A.st_area + g, cnt[i]);
            atomicMin(A.st_x0 + g, tc.x0 + __builtin_ctz(cmask[i]));
            atomicMax(A.st_x1 + g, tc.x0 + 31 - __builtin_clz(cmask[i]));
            atomicMin(A.st_y0 + g, tc.y0 + __builtin_ctz(rmask[i]));
            atomicMax(A.st_y1 + g, tc.y0 + 31 - __builtin_clz(rmask[i]));
        }
        if (A.obj_list && g == pix_id(A, tc, i)) A.obj_list[atomicAdd(A.n_obj, 1)] = g;
    }
}

int launch_ccl(const CclArgs &a, hipStream_t s) {
    if (a.pred == CclPred::Level && (a.n_levels < 1 || a.n_levels > MAXLEV)) {
        set_error("ccl: bad level count %d", a.n_levels);
        return RT_EINVAL;
    }
    const int ntx = (a.w + TW - 1) / TW, nty = (a.h + TH - 1) / TH;
    const int nlev = a.pred == CclPred::Level ? a.n_levels : 1;
    const int64_t nid = (int64_t)a.w * a.h + 1;
    // the virtual node id 0 of every level is its own root
    for (int l = 0; l < nlev; ++l) {
        int e = launch_fill_i32(a.ids + l * nid, 0, 1, s);
        if (e) return e;
    }
    hipLaunchKernelGGL(k_ccl_local, dim3(ntx * nty), dim3(NT), 0, s, a);
    RT_HIP(hipGetLastError());
    int64_t n_vert = (int64_t)(ntx - 1) * a.h;
    int64_t n_pairs = n_vert + (int64_t)(nty - 1) * a.w;
    if (n_pairs > 0) {
        hipLaunchKernelGGL(k_ccl_merge, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s, a, n_vert);
        RT_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ccl_flatten, dim3(ntx * nty), dim3(NT), 0, s, a);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rtseg
