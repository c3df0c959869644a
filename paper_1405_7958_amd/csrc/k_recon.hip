// Grayscale reconstruction by dilation -- the irregular wavefront propagation
// (IWPP) behind ReconToNuclei (Sec. 5.1).
//
// The paper's GPU version keeps a queue of active pixels; here the unit of
// activity is a 64 x 64 tile handled by one wavefront:
//   * the tile's current values live in 64 VGPRs per lane (lane = column),
//     the mask in LDS;
//   * a sweep is four directional scans: down and up with lane = column, then
//     (after a transpose through LDS) right and left with lane = row.  Each
//     scan step takes the 3 neighbours of the previous row/column from the
//     lane's own register and its two neighbour lanes via DPP wave shifts,
//     so a value can travel 64 pixels in one scan;
//   * sweeps repeat until the tile reaches its local fixpoint; values of the
//     one-pixel halo come from the neighbouring tiles as they are in memory;
//   * a tile whose edge changed puts the neighbours that read that edge on
//     the next round's worklist (deduplicated by a per-tile stamp).
// Rounds run until the worklist is empty.  Updates only ever raise values to
// something at most the final result, so reading a neighbour's edge while it
// is being rewritten is harmless: the neighbour re-queues the tile if its
// edge changed after the read.
#include "rt_internal.h"

#include <climits>

namespace rtseg {

constexpr int RTILE = 64;
constexpr int NEG = INT_MIN;

struct RoundArgs {
    const void *mask;
    void *r;
    const uint8_t *domain;
    int w, h;
    int64_t pitch;
    int ntx, nty;
    const int32_t *list_in;
    int32_t *list_out;
    int32_t *cnt;        // 3 rotating counters
    int k;               // round index
    int first;           // 1: process every tile
    uint32_t *stamp;
    uint32_t epoch;      // stamp value of this round's output list
    int max_sweeps;
};

__device__ __forceinline__ int shr1(int v, int old) {  // lane i <- lane i-1; lane 0 <- old
    return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int shl1(int v, int old) {  // lane i <- lane i+1; lane 63 <- old
    return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}

template <typename T>
__device__ __forceinline__ int gval(const RoundArgs &a, const T *p, int x, int y) {
    if (x < 0 || y < 0 || x >= a.w || y >= a.h) return NEG;
    int64_t o = (int64_t)y * a.pitch + x;
    if (a.domain && !a.domain[o]) return NEG;
    return (int)p[o];
}

__device__ __forceinline__ bool wave_any(bool c) { return __ballot(c) != 0; }

// One directional scan over the 64 rows held in r[] (lane = column).
// prev*: values of the row before the first one; edgeL/edgeR: the halo
// column values used by lanes 0 / 63 for each row.
template <int CONN, bool DOWN>
__device__ __forceinline__ bool scan_v(int (&r)[64], const int (*Is)[65], int lane, int pc, int pl, int pr,
                                       const int *edgeL, const int *edgeR) {
    bool ch = false;
#pragma unroll
    for (int s = 0; s < 64; ++s) {
        const int y = DOWN ? s : 63 - s;
        int m = pc;
        if (CONN == 8) m = max(m, max(pl, pr));
        int iv = Is[y][lane];
        int nv = max(r[y], min(m, iv));
        ch |= nv != r[y];
        r[y] = nv;
        pc = nv;
        if (CONN == 8) {
            pl = shr1(nv, edgeL[y]);
            pr = shl1(nv, edgeR[y]);
        }
    }
    return ch;
}

template <typename T, int CONN>
__global__ __launch_bounds__(64) void k_recon_round(RoundArgs a) {
    const int lane = threadIdx.x;
    int32_t *cnt_in = a.cnt + (a.k % 3);
    int32_t *cnt_out = a.cnt + ((a.k + 1) % 3);
    int32_t *cnt_clr = a.cnt + ((a.k + 2) % 3);
    if (blockIdx.x == 0 && lane == 0) *cnt_clr = 0;
    const int ntiles = a.ntx * a.nty;
    const int n_in = a.first ? ntiles : *cnt_in;
    if ((int)blockIdx.x >= n_in) return;
    const int tile = a.first ? (int)blockIdx.x : a.list_in[blockIdx.x];
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int x0 = tx * RTILE, y0 = ty * RTILE;
    const T *mask = static_cast<const T *>(a.mask);
    T *rr = static_cast<T *>(a.r);

    __shared__ int Is[64][65];
    __shared__ int Ts[64][65];
    __shared__ int hT[66], hB[66], hL[64], hR[64];
    __shared__ int oL[64], oR[64];

    int r[64];
    const int x = x0 + lane;
#pragma unroll
    for (int y = 0; y < 64; ++y) {
        r[y] = gval<T>(a, rr, x, y0 + y);
        Is[y][lane] = gval<T>(a, mask, x, y0 + y);
    }
    hT[lane + 1] = gval<T>(a, rr, x, y0 - 1);
    hB[lane + 1] = gval<T>(a, rr, x, y0 + 64);
    if (lane == 0) {
        hT[0] = gval<T>(a, rr, x0 - 1, y0 - 1);
        hB[0] = gval<T>(a, rr, x0 - 1, y0 + 64);
        hT[65] = gval<T>(a, rr, x0 + 64, y0 - 1);
        hB[65] = gval<T>(a, rr, x0 + 64, y0 + 64);
    }
    hL[lane] = gval<T>(a, rr, x0 - 1, y0 + lane);
    hR[lane] = gval<T>(a, rr, x0 + 64, y0 + lane);
    const int oT = r[0], oB = r[63];
#pragma unroll
    for (int y = 0; y < 64; ++y) Ts[y][lane] = r[y];
    __syncthreads();
    oL[lane] = Ts[lane][0];
    oR[lane] = Ts[lane][63];
    __syncthreads();

    bool any_change = false;
    bool converged = false;
    for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
        bool ch = false;
        // down / up, lane = column
        ch |= scan_v<CONN, true>(r, Is, lane, hT[lane + 1], hT[lane], hT[lane + 2], hL, hR);
        ch |= scan_v<CONN, false>(r, Is, lane, hB[lane + 1], hB[lane], hB[lane + 2], hL, hR);
        // transpose: lane = row
#pragma unroll
        for (int y = 0; y < 64; ++y) Ts[y][lane] = r[y];
        __syncthreads();
#pragma unroll
        for (int xx = 0; xx < 64; ++xx) r[xx] = Ts[lane][xx];
        __syncthreads();
        // right / left: previous column comes from the left/right halo
        {
            bool c2 = false;
            int pc = hL[lane];
            int pl = lane > 0 ? hL[lane - 1] : hT[0];
            int pr = lane < 63 ? hL[lane + 1] : hB[0];
#pragma unroll
            for (int xx = 0; xx < 64; ++xx) {
                int m = pc;
                if (CONN == 8) m = max(m, max(pl, pr));
                int nv = max(r[xx], min(m, Is[lane][xx]));
                c2 |= nv != r[xx];
                r[xx] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr1(nv, hT[xx + 1]);
                    pr = shl1(nv, hB[xx + 1]);
                }
            }
            pc = hR[lane];
            pl = lane > 0 ? hR[lane - 1] : hT[65];
            pr = lane < 63 ? hR[lane + 1] : hB[65];
#pragma unroll
            for (int s = 0; s < 64; ++s) {
                const int xx = 63 - s;
                int m = pc;
                if (CONN == 8) m = max(m, max(pl, pr));
                int nv = max(r[xx], min(m, Is[lane][xx]));
                c2 |= nv != r[xx];
                r[xx] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr1(nv, hT[xx + 1]);
                    pr = shl1(nv, hB[xx + 1]);
                }
            }
            ch |= c2;
        }
        // transpose back: lane = column
#pragma unroll
        for (int xx = 0; xx < 64; ++xx) Ts[lane][xx] = r[xx];
        __syncthreads();
#pragma unroll
        for (int y = 0; y < 64; ++y) r[y] = Ts[y][lane];
        __syncthreads();
        if (!wave_any(ch)) {
            converged = true;
            break;
        }
        any_change = true;
    }
    if (!any_change) return;

    // write back (own column), only real graph nodes
#pragma unroll
    for (int y = 0; y < 64; ++y) {
        int gy = y0 + y;
        if (x < a.w && gy < a.h && r[y] != NEG) {
            int64_t o = (int64_t)gy * a.pitch + x;
            rr[o] = (T)r[y];
        }
    }
    // which edges changed?  (Ts holds the final tile, row-major)
    const bool cT = r[0] != oT, cB = r[63] != oB;
    const bool cL = Ts[lane][0] != oL[lane], cR = Ts[lane][63] != oR[lane];
    const uint64_t mT = __ballot(cT), mB = __ballot(cB), mL = __ballot(cL), mR = __ballot(cR);
    if (lane == 0) {
        int nb[8];
        int nn = 0;
        auto add = [&](int dx, int dy) {
            int nx = tx + dx, ny = ty + dy;
            if (nx >= 0 && ny >= 0 && nx < a.ntx && ny < a.nty) nb[nn++] = ny * a.ntx + nx;
        };
        if (mT) add(0, -1);
        if (mB) add(0, 1);
        if (mL) add(-1, 0);
        if (mR) add(1, 0);
        if (CONN == 8) {
            if (mT & 1ull) add(-1, -1);
            if (mT >> 63) add(1, -1);
            if (mB & 1ull) add(-1, 1);
            if (mB >> 63) add(1, 1);
        }
        if (!converged) nb[nn++] = tile;  // sweep budget exhausted: continue next round
        for (int k = 0; k < nn; ++k) {
            if (atomicExch(a.stamp + nb[k], a.epoch) != a.epoch) a.list_out[atomicAdd(cnt_out, 1)] = nb[k];
        }
    }
}

// R0 = min(marker, mask) (out may alias marker)
template <typename T>
__global__ void k_recon_init(const T *marker, const T *mask, T *out, int w, int h, int64_t pitch) {
    int64_t n = (int64_t)w * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = i / w, x = i - y * w;
        int64_t o = y * pitch + x;
        T a = marker[o], b = mask[o];
        out[o] = a < b ? a : b;
    }
}

int recon_init(int dtype, const void *marker, const void *mask, void *out, const uint8_t *, int w, int h,
               int64_t pitch, hipStream_t s) {
    int64_t n = (int64_t)w * h;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (dtype == RT_U8)
        hipLaunchKernelGGL(k_recon_init<uint8_t>, dim3(grid), dim3(256), 0, s, (const uint8_t *)marker,
                           (const uint8_t *)mask, (uint8_t *)out, w, h, pitch);
    else
        hipLaunchKernelGGL(k_recon_init<int32_t>, dim3(grid), dim3(256), 0, s, (const int32_t *)marker,
                           (const int32_t *)mask, (int32_t *)out, w, h, pitch);
    return hip_fail(hipGetLastError(), "k_recon_init");
}

// Level choice for the connectivity lower bound: the smallest levels whose
// upper-set density drops to each of the target fractions (the bound helps
// most around the density at which the upper set stops percolating).
__global__ void k_select_levels(const uint32_t *hist, int n_levels, int32_t *levels) {
    if (threadIdx.x != 0) return;
    const double q[8] = {0.80, 0.70, 0.60, 0.52, 0.46, 0.41, 0.36, 0.30};
    double total = 0;
    for (int v = 0; v < 256; ++v) total += hist[v];
    double above = total;  // pixels with value >= v
    int k = 0;
    for (int v = 0; v < 256 && k < n_levels; ++v) {
        while (k < n_levels && above <= q[k] * total) levels[k++] = v > 0 ? v : 1;
        above -= hist[v];
    }
    while (k < n_levels) levels[k++] = 255;
}

int launch_select_levels(const uint32_t *hist, int n_levels, int32_t *levels, hipStream_t s) {
    hipLaunchKernelGGL(k_select_levels, dim3(1), dim3(64), 0, s, hist, n_levels, levels);
    return hip_fail(hipGetLastError(), "k_select_levels");
}

template <typename T, int CONN>
static void launch_round(const RoundArgs &ra, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_recon_round<T, CONN>), dim3(grid), dim3(64), 0, s, ra);
}

int recon_rounds(rt_ctx_impl *c, const ReconArgs &a, hipStream_t s) {
    const int ntx = (a.w + RTILE - 1) / RTILE, nty = (a.h + RTILE - 1) / RTILE;
    const int ntiles = ntx * nty;
    int e = ensure_stamps(c, (size_t)ntiles);
    if (e) return e;
    const size_t mark = c->arena.off;
    int32_t *lists = (int32_t *)c->arena.take(sizeof(int32_t) * (2 * (size_t)ntiles + 4));
    if (!lists) {
        c->arena.off = mark;
        set_error("recon: scratch arena too small");
        return RT_ENOMEM;
    }
    int32_t *cnt = lists + 2 * ntiles;
    RoundArgs ra;
    ra.mask = a.mask;
    ra.r = a.r;
    ra.domain = a.domain;
    ra.w = a.w;
    ra.h = a.h;
    ra.pitch = a.pitch;
    ra.ntx = ntx;
    ra.nty = nty;
    ra.cnt = cnt;
    ra.stamp = c->stamps;
    ra.max_sweeps = c->knobs.recon_max_sweeps;
    int k = 0;
    const int batch = c->knobs.recon_round_batch;
    const int max_rounds = 4 * (ntx + nty) * (int)std::max(1, 4096 / std::max(1, ra.max_sweeps)) + 64;
    e = RT_OK;
    for (;;) {
        for (int b = 0; b < batch; ++b, ++k) {
            ra.k = k;
            ra.first = k == 0;
            ra.list_in = lists + (k & 1) * ntiles;
            ra.list_out = lists + ((k + 1) & 1) * ntiles;
            if (++c->stamp_epoch == 0) {
                RT_HIP(hipMemsetAsync(c->stamps, 0, sizeof(uint32_t) * c->stamps_cap, s));
                c->stamp_epoch = 1;
            }
            ra.epoch = c->stamp_epoch;
            if (k == 0) RT_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * 3, s));
            if (a.dtype == RT_U8) {
                if (a.conn == 8) launch_round<uint8_t, 8>(ra, ntiles, s);
                else launch_round<uint8_t, 4>(ra, ntiles, s);
            } else {
                if (a.conn == 8) launch_round<int32_t, 8>(ra, ntiles, s);
                else launch_round<int32_t, 4>(ra, ntiles, s);
            }
            RT_HIP(hipGetLastError());
        }
        // the list produced by the last round: counter (k % 3)
        RT_HIP(hipMemcpyAsync(c->pinned, cnt + (k % 3), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        RT_HIP(hipStreamSynchronize(s));
        if (c->pinned[0] == 0) break;
        if (k > max_rounds) {
            set_error("recon: no convergence after %d rounds", k);
            e = RT_EDEVICE;
            break;
        }
    }
    c->arena.off = mark;
    return e;
}

}  // namespace rtseg
