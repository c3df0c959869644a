// Grayscale reconstruction by dilation -- the irregular wavefront propagation
// (IWPP) behind ReconToNuclei (Sec. 5.1).
//
// The paper's GPU version keeps a queue of active pixels; here the unit of
// activity is a 62 x 62 tile handled by one wavefront:
//   * the wave holds the tile and its one-pixel ring of neighbour values as a
//     64 x 64 block, 64 registers per lane, with the mask in registers too
//     (both orientations, packed for uint8), so a scan step touches no memory
//     and ring lanes feed the DPP shifts like any other lane;
//   * a sweep is four directional scans: down and up with lane = column, then
//     (after an LDS transpose) right and left with lane = row.  Each scan step
//     takes the 3 neighbours of the previous row/column from the lane's own
//     register and its two neighbour lanes via DPP wave shifts, so a value can
//     travel 64 pixels in one scan;
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

constexpr int RIN = 62;   // interior edge of a tile (the 64-lane block adds a 1-px ring)
constexpr int NEG = INT_MIN;

struct RoundArgs {
    const ReconImg *imgs;  // one record per image (device)
    int n;
    int total;           // tiles of the whole batch
    const int32_t *list_in;
    int32_t *list_out;
    int32_t *cnt;        // 3 rotating counters
    int k;               // round index
    int first;           // 1: process every tile
    uint32_t *stamp;
    uint32_t epoch;      // stamp value of this round's output list
    int max_sweeps;
    unsigned long long *visits;   // nullable: tiles processed (stage timing only)
};

__device__ __forceinline__ int recon_img_of(const ReconImg *imgs, int n, int u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].unit0 <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}


template <typename T>
__device__ __forceinline__ int gval(const ReconImg &a, const T *p, int x, int y) {
    if (x < 0 || y < 0 || x >= a.w || y >= a.h) return NEG;
    int64_t o = (int64_t)y * a.pitch + x;
    if (a.domain && !a.domain[o]) return NEG;
    return (int)p[o];
}

__device__ __forceinline__ bool wave_any(bool c) { return __ballot(c) != 0; }

// The mask of one tile in registers, for one orientation (64 entries per
// lane).  uint8 masks are packed four per register; non-members (outside the
// image or the domain) read as NEG, so they neither rise nor propagate.
template <typename T>
struct MaskRegs;
template <>
struct MaskRegs<uint8_t> {
    uint32_t p[16];
    uint64_t mem;
    __device__ void clear() {
#pragma unroll
        for (int k = 0; k < 16; ++k) p[k] = 0;
        mem = 0;
    }
    __device__ void set(int k, int v) {  // k compile-time after unrolling
        if (v != NEG) {
            p[k >> 2] |= (uint32_t)(v & 255) << ((k & 3) * 8);
            mem |= 1ull << k;
        }
    }
    __device__ int eff(int k) const { return ((mem >> k) & 1ull) ? (int)((p[k >> 2] >> ((k & 3) * 8)) & 255u) : NEG; }
};
template <>
struct MaskRegs<int32_t> {
    int v[64];
    __device__ void clear() {}
    __device__ void set(int k, int x) { v[k] = x; }
    __device__ int eff(int k) const { return v[k]; }
};

// one scan step: value of this pixel given the three predecessors' maximum m
__device__ __forceinline__ int step_val(int rv, int m, int mv) { return max(rv, min(m, mv)); }
// the median of three (one v_med3 instruction): step_val(a, b, c) when a <= c
__device__ __forceinline__ int med3(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

__device__ __forceinline__ int shr0(int v) {  // lane i <- lane i-1 (lane 0: don't care)
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int shl0(int v) {  // lane i <- lane i+1 (lane 63: don't care)
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
}

template <typename T, int CONN, bool QUEUE, typename Push>
__device__ void recon_tile(const ReconImg &a, int gtile, int max_sweeps, int (*Ts)[65], Push push);

// Plain uint8 images (no domain), the reconstruction of ReconToNuclei.
//
// Every value is >= 0 here, so a pixel outside the image carries the value 0
// and the mask 0: for it max(r, min(m, 0)) = r, so it never changes, and the
// zeros it feeds to its neighbours' scan steps never raise a member, whose
// value is >= 0.  Every other position of the block, the ring included,
// carries its mask: values start at min(marker, mask) and never pass the
// mask, so value <= mask holds everywhere and a scan step
// max(r, min(m, mask)) is the median of the three (one instruction).  A ring
// pixel may then rise in the registers; it rises only to a value its own
// reconstruction reaches too (the neighbours it takes from hold lower bounds
// of theirs), so the interior stays a lower bound of the result, the ring's
// registers are never written back, and at the fixpoint of the whole image
// no ring pixel rises.  Scan steps need no membership test.  Both images are staged
// through LDS in row order: each lane loads 17 aligned dwords per image (the
// 64-byte rows of a block start at any byte), each clamped to a dword that
// holds at least one byte of its row; an aligned dword never crosses a page,
// so no load leaves the pages of the row's bytes.  Bytes outside the image
// are masked when the registers are built.  The sweep tests convergence by
// the wave's sum of values: values only rise, so a sweep changed something
// iff the sum grew.
constexpr int SP = 68;                   // staging row pitch in bytes (17 dwords)
constexpr int TP = 66;                   // transpose row pitch in uint16 (33 dwords)
constexpr int PLAIN_LDS = 2 * 64 * SP;   // two staged images; >= 64 * TP * 2

extern "C" __device__ int __ockl_wfred_add_i32(int);

// bytes b of a dword whose index 4k + b lies in [lo, hi]
__device__ __forceinline__ uint32_t byte_span(int k, int lo, int hi) {
    const int a = min(max(lo - 4 * k, 0), 4), b = min(max(hi + 1 - 4 * k, 0), 4);
    return (uint32_t)(((1ull << (8 * b)) - 1ull) & ~((1ull << (8 * a)) - 1ull));
}

template <int CONN, bool QUEUE, typename Push>
__device__ void recon_tile_plain(const ReconImg &a, int gtile, int max_sweeps, uint8_t *lds, Push push) {
    const int lane = threadIdx.x;
    const int tile = gtile - a.unit0;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    // block coordinate (i, j) is image pixel (x0-1+i, y0-1+j)
    const int x0 = tx * RIN, y0 = ty * RIN;
    uint8_t *rr = static_cast<uint8_t *>(a.r);
    const uintptr_t bR = (uintptr_t)rr, bM = (uintptr_t)a.mask;
    uint8_t *sR = lds, *sM = lds + 64 * SP;
    uint16_t *Tw = reinterpret_cast<uint16_t *>(lds);
    // last interior column / row inside the image (block coordinates)
    const int limw = min(RIN, a.w - x0), limh = min(RIN, a.h - y0);

    // byte offsets from the dword-aligned image bases (the host keeps the
    // images below 2 GiB for this path)
    const uintptr_t bR4 = bR & ~(uintptr_t)3, bM4 = bM & ~(uintptr_t)3;
    const int aR = (int)(bR & 3), aM = (int)(bM & 3);
    const int pitch = (int)a.pitch;
    {
        typedef const __attribute__((address_space(1))) uint32_t *gw;
        typedef const __attribute__((address_space(1))) uint8_t *gb;
        const gb gR = (gb)bR4, gM = (gb)bM4;
        // the lane index, opaque to the optimiser so that the addresses below
        // are recomputed per tile rather than held in registers across tiles
        int ln = lane;
        asm volatile("" : "+v"(ln));
        // dwords 0..15 of rows 4k .. 4k+3 (16 lanes per row), then dword 16
        // of row `lane`
        const int lr = ln >> 4, ld = ln & 15;
        uint32_t vr[17], vm[17];
#pragma unroll
        for (int k = 0; k < 17; ++k) {
            const int row = k < 16 ? 4 * k + lr : ln, d = k < 16 ? ld : 16;
            const int yo = min(max(y0 - 1 + row, 0), a.h - 1) * pitch;
            const int sr = aR + yo, sm = aM + yo;   // the row's first byte
            const int orr = min(max(((sr + x0 - 1) & ~3) + 4 * d, sr & ~3), (sr + a.w - 1) & ~3);
            const int om = min(max(((sm + x0 - 1) & ~3) + 4 * d, sm & ~3), (sm + a.w - 1) & ~3);
            vr[k] = *(gw)(gR + (uint32_t)orr);
            vm[k] = *(gw)(gM + (uint32_t)om);
            // addresses are computed next to their loads
            __builtin_amdgcn_sched_barrier(0);
        }
        uint32_t *dR = reinterpret_cast<uint32_t *>(sR + lr * SP + 4 * ld);
        uint32_t *dM = reinterpret_cast<uint32_t *>(sM + lr * SP + 4 * ld);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            dR[k * SP] = vr[k];   // (4k + lr) * SP bytes = k * SP dwords further
            dM[k * SP] = vm[k];
        }
        reinterpret_cast<uint32_t *>(sR + ln * SP)[16] = vr[16];
        reinterpret_cast<uint32_t *>(sM + ln * SP)[16] = vm[16];
    }
    __syncthreads();

    const int gx = x0 - 1 + lane;
    const bool col_ok = gx >= 0 && gx < a.w;
    const bool col_m = lane >= 1 && lane <= limw;
    const bool row_m = lane >= 1 && lane <= limh;
    const bool edge = x0 == 0 || y0 == 0 || x0 + RIN >= a.w || y0 + RIN >= a.h;
    const uint32_t colmask = col_m ? ~0u : 0u, rowmask = row_m ? ~0u : 0u;
    // the masks of every position inside the image, the ring included (rows
    // and columns outside the image: 0)
    const int gyl = y0 - 1 + lane;
    const uint32_t colimg = col_ok ? ~0u : 0u, rowimg = (gyl >= 0 && gyl < a.h) ? ~0u : 0u;
    const int jlo = y0 == 0 ? 1 : 0, jhi = min(63, a.h - y0);
    const int clo = x0 == 0 ? 1 : 0, chi = min(63, a.w - x0);
    int r[64];
    uint32_t mc[16], mr[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        uint32_t p = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = 4 * k + b;
            const int yo = min(max(y0 - 1 + j, 0), a.h - 1) * pitch;
            const int oR = (aR + yo + x0 - 1) & 3, oM = (aM + yo + x0 - 1) & 3;
            r[j] = sR[j * SP + oR + lane];
            p |= (uint32_t)sM[j * SP + oM + lane] << (8 * b);
        }
        mc[k] = p & byte_span(k, jlo, jhi) & colimg;
        // at most eight LDS reads in flight: the counter holds no more anyway
        __builtin_amdgcn_sched_barrier(0);
    }
    if (edge) {
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const int gy = y0 - 1 + j;
            r[j] = (col_ok && gy >= 0 && gy < a.h) ? r[j] : 0;
        }
    }
    // lane = row: the mask's row, the original values of columns 1 and 62,
    // and those of the ring columns 0 and 63 (0 outside the image)
    int oL, oR, oL0, oR0;
    {
        const int yo = min(max(y0 - 1 + lane, 0), a.h - 1) * pitch;
        const int o = (aM + yo + x0 - 1) & 3, orr = (aR + yo + x0 - 1) & 3;
        const uint32_t *srow = reinterpret_cast<const uint32_t *>(sM + lane * SP);
        uint32_t dw[17];
#pragma unroll
        for (int d = 0; d < 17; ++d) dw[d] = srow[d];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            mr[k] = __builtin_amdgcn_alignbyte(dw[k + 1], dw[k], o) & byte_span(k, clo, chi) & rowimg;
        oL = (int)((uint32_t)sR[lane * SP + orr + 1] & rowmask);
        oR = (int)((uint32_t)sR[lane * SP + orr + RIN] & (limw >= RIN ? rowmask : 0u));
        oL0 = (int)((uint32_t)sR[lane * SP + orr] & (x0 > 0 ? rowimg : 0u));
        oR0 = (int)((uint32_t)sR[lane * SP + orr + 63] & (x0 + RIN < a.w ? rowimg : 0u));
    }
    const int oT = r[1], oB = r[62];
    const int oT0 = r[0], oB0 = r[63];   // the ring rows as loaded
    int tot0 = 0;
#pragma unroll
    for (int j = 0; j < 64; ++j) tot0 += r[j];
    int prev = __ockl_wfred_add_i32(tot0);
    __syncthreads();   // the staging area becomes the transpose buffer

    bool any_change = false;
    bool converged = false;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // down and up, lane = column
        {
            int pc = r[0];
#pragma unroll
            for (int j = 1; j < 64; ++j) {
                const int m = CONN == 8 ? max(pc, max(shr0(pc), shl0(pc))) : pc;
                pc = med3(r[j], m, (int)((mc[j >> 2] >> (8 * (j & 3))) & 255u));
                r[j] = pc;
            }
#pragma unroll
            for (int j = 62; j >= 0; --j) {
                const int m = CONN == 8 ? max(pc, max(shr0(pc), shl0(pc))) : pc;
                pc = med3(r[j], m, (int)((mc[j >> 2] >> (8 * (j & 3))) & 255u));
                r[j] = pc;
            }
        }
#pragma unroll
        for (int j = 0; j < 64; ++j) Tw[j * TP + lane] = (uint16_t)r[j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 64; ++i) r[i] = Tw[lane * TP + i];
        __syncthreads();
        // right and left, lane = row; the left scan also sums the final values
        int acc;
        {
            int pc = r[0];
#pragma unroll
            for (int i = 1; i < 64; ++i) {
                const int m = CONN == 8 ? max(pc, max(shr0(pc), shl0(pc))) : pc;
                pc = med3(r[i], m, (int)((mr[i >> 2] >> (8 * (i & 3))) & 255u));
                r[i] = pc;
            }
            acc = pc;
#pragma unroll
            for (int i = 62; i >= 0; --i) {
                const int m = CONN == 8 ? max(pc, max(shr0(pc), shl0(pc))) : pc;
                pc = med3(r[i], m, (int)((mr[i >> 2] >> (8 * (i & 3))) & 255u));
                r[i] = pc;
                acc += pc;
            }
        }
#pragma unroll
        for (int i = 0; i < 64; ++i) Tw[lane * TP + i] = (uint16_t)r[i];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 64; ++j) r[j] = Tw[j * TP + lane];
        __syncthreads();
        const int tot = __ockl_wfred_add_i32(acc);
        if (tot == prev) {
            converged = true;
            break;
        }
        prev = tot;
        any_change = true;
    }
    if (!any_change) return;

    // write back the interior members (own column)
    if (col_m) {
#pragma unroll
        for (int j = 1; j < 63; ++j)
            if (j <= limh) rr[(int64_t)(y0 - 1 + j) * a.pitch + gx] = (uint8_t)r[j];
    }
    // which interior edges changed?  (Tw keeps the row-major copy)
    const bool cT = col_m && r[1] != oT, cB = col_m && r[62] != oB;
    const bool cL = row_m && (int)Tw[lane * TP + 1] != oL, cR = row_m && (int)Tw[lane * TP + RIN] != oR;
    const uint64_t mT = __ballot(cT), mB = __ballot(cB), mL = __ballot(cL), mR = __ballot(cR);
    // neighbours to visit: a side whose edge changed; with 8-connectivity a
    // diagonal neighbour when the interior corner next to it changed
    bool pT = mT != 0, pB = mB != 0, pL = mL != 0, pR = mR != 0;
    bool pTL = (mT >> 1) & 1ull, pTR = (mT >> 62) & 1ull, pBL = (mB >> 1) & 1ull, pBR = (mB >> 62) & 1ull;
    if (converged) {
        // The ring pixels rose in registers to every value this tile's pixels
        // can give them (the block is at its fixpoint), so a neighbour whose
        // ring pixels all kept their loaded values, which are at most its
        // current ones, has nothing to gain from this tile.  A neighbour is
        // visited when an edge pixel next to it changed and one of its ring
        // pixels rose; an unchanged edge pixel gave its value at an earlier
        // visit, which queued the neighbour then if it needed it.  (Without
        // convergence the ring values are not final: every changed side
        // counts.)
        const uint64_t uT = __ballot(r[0] > oT0), uB = __ballot(r[63] > oB0);
        const uint64_t uL = __ballot((int)Tw[lane * TP] > oL0), uR = __ballot((int)Tw[lane * TP + 63] > oR0);
        const uint64_t mid = ~1ull & ~(1ull << 63);   // ring positions 1..62 belong to the side's neighbour
        pT = pT && (uT & mid);
        pB = pB && (uB & mid);
        pL = pL && (uL & mid);
        pR = pR && (uR & mid);
        pTL = pTL && (uT & 1ull);
        pTR = pTR && (uT >> 63);
        pBL = pBL && (uB & 1ull);
        pBR = pBR && (uB >> 63);
    }
    if constexpr (QUEUE) __threadfence();   // release the tile's writes before announcing them
    int nb[9];
    int nn = 0;
    auto add = [&](int dx, int dy) {
        int nx = tx + dx, ny = ty + dy;
        if (nx >= 0 && ny >= 0 && nx < a.ntx && ny < a.nty) nb[nn++] = a.unit0 + ny * a.ntx + nx;
    };
    if (pT) add(0, -1);
    if (pB) add(0, 1);
    if (pL) add(-1, 0);
    if (pR) add(1, 0);
    if (CONN == 8) {
        if (pTL) add(-1, -1);
        if (pTR) add(1, -1);
        if (pBL) add(-1, 1);
        if (pBR) add(1, 1);
    }
    if (!converged) nb[nn++] = gtile;
    int mine = -1;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (k == lane && k < nn) mine = nb[k];
    push(mine, lane < nn);
}

template <typename T, int CONN, bool PLAIN>
__global__ __launch_bounds__(64, PLAIN ? 2 : 1) void k_recon_round(RoundArgs ra) {
    __shared__ __align__(16) uint8_t lds[PLAIN ? PLAIN_LDS : 64 * 65 * 4];
    const int lane = threadIdx.x;
    int32_t *cnt_in = ra.cnt + (ra.k % 3);
    int32_t *cnt_out = ra.cnt + ((ra.k + 1) % 3);
    int32_t *cnt_clr = ra.cnt + ((ra.k + 2) % 3);
    if (blockIdx.x == 0 && lane == 0) *cnt_clr = 0;
    const int n_in = ra.first ? ra.total : *cnt_in;
    if (ra.visits && lane == 0 && blockIdx.x == 0) atomicAdd(ra.visits, (unsigned long long)n_in);
    for (int slot = blockIdx.x; slot < n_in; slot += gridDim.x) {
        // the first round visits every tile: consecutive workgroups go to the
        // eight XCDs in turn, so slot s takes a tile of the s % 8-th eighth of
        // the tile range, and tiles that share halo rows share an L2
        int gtile;
        if (ra.first) {
            const int q = ra.total >> 3, rem = ra.total & 7, x = slot & 7;
            gtile = x * q + min(x, rem) + (slot >> 3);
        } else {
            gtile = ra.list_in[slot];
        }
        const ReconImg a = ra.imgs[recon_img_of(ra.imgs, ra.n, gtile)];
        // every lane calls push; one counter update per wave for its new entries
        auto push = [&](int item, bool valid) {
            const bool fresh = valid && atomicExch(ra.stamp + item, ra.epoch) != ra.epoch;
            const uint64_t m = __ballot(fresh);
            if (!m) return;
            int base = 0;
            if (lane == 0) base = atomicAdd(cnt_out, __popcll(m));
            base = __shfl(base, 0, 64);
            if (fresh) ra.list_out[base + __popcll(m & ((1ull << lane) - 1))] = item;
        };
        if constexpr (PLAIN)
            recon_tile_plain<CONN, false>(a, gtile, ra.max_sweeps, lds, push);
        else
            recon_tile<T, CONN, false>(a, gtile, ra.max_sweeps, reinterpret_cast<int (*)[65]>(lds), push);
        __syncthreads();
    }
}

// Work-queue variant: one persistent launch in which every wave takes a
// ticket, waits for the tile pushed under that ticket, processes it and
// pushes the neighbours its change reaches.  inq holds a tile's state: 0 idle,
// 1 queued, 2 in a visit, 3 in a visit and pushed meanwhile.  Only an idle
// tile enters the queue, and a tile pushed during its visit enters it again
// when that visit ends, so no two visits of one tile overlap (an older visit
// finishing last would write back values below the newer one's).  `pending` counts tiles pushed and not yet finished; the waves
// leave when it reaches zero.  A waiting wave that sees no tile finished
// anywhere for spin_limit wall-clock ticks (a stall: one tile visit takes far
// less) raises `abort` and leaves; the host then finishes with ordinary
// rounds, which accept any intermediate state.
struct QueueArgs {
    const ReconImg *imgs;
    int n, total;
    unsigned long long *ring;   // 2*total entries: ticket << 32 | tile
    unsigned int *ctl;          // head, tail, pending, abort, finished
    unsigned int *inq;
    int max_sweeps;
    long long spin_limit;
    unsigned long long *visits; // nullable
};

constexpr unsigned long long RING_EMPTY = ~0ull;

template <typename T, int CONN, bool PLAIN>
__global__ __launch_bounds__(64, PLAIN ? 2 : 1) void k_recon_queue(QueueArgs q) {
    __shared__ __align__(16) uint8_t lds[PLAIN ? PLAIN_LDS : 64 * 65 * 4];
    const int lane = threadIdx.x;
    const unsigned cap = 2u * (unsigned)q.total;
    unsigned int *head = q.ctl, *tail = q.ctl + 1, *pending = q.ctl + 2, *abortf = q.ctl + 3, *done = q.ctl + 4;
    for (;;) {
        int item = -1;
        if (lane == 0) {
            const unsigned t = atomicAdd(head, 1u);
            const unsigned slot = t % cap;
            long long t0 = wall_clock64();
            unsigned seen = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (unsigned spin = 0;; ++spin) {
                const unsigned long long e =
                    __hip_atomic_load(q.ring + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(e >> 32) == t) {
                    item = (int)(e & 0xffffffffull);
                    break;
                }
                // the shared counters are polled less often than the own slot
                if (spin & 7u) {
                    __builtin_amdgcn_s_sleep(8);
                    continue;
                }
                if (__hip_atomic_load(pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                    item = -2;
                    break;
                }
                const unsigned now_done = __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (now_done != seen) {   // progress elsewhere: restart the stall timer
                    seen = now_done;
                    t0 = wall_clock64();
                } else if (wall_clock64() - t0 > q.spin_limit) {
                    atomicExch(abortf, 1u);
                    item = -2;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        item = __shfl(item, 0, 64);
        if (item < 0) break;
        if (lane == 0) {
            atomicExch(q.inq + item, 2u);   // queued -> in a visit
            if (q.visits) atomicAdd(q.visits, 1ull);
        }
        // acquire after leaving the queue: a neighbour that changed this
        // tile's input and found it still queued (so did not queue it again)
        // released its writes before that test, which precedes the exchange
        // above; fencing before the exchange could keep stale lines cached
        __threadfence();
        const ReconImg a = q.imgs[recon_img_of(q.imgs, q.n, item)];
        auto enqueue = [&](int nb) {
            atomicAdd(pending, 1u);
            const unsigned t = atomicAdd(tail, 1u);
            __hip_atomic_store(q.ring + t % cap, ((unsigned long long)t << 32) | (unsigned)nb, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        };
        auto push = [&](int nb, bool valid) {
            if (!valid) return;
            // idle -> queued (enqueue), in a visit -> pushed meanwhile; a
            // queued or already marked tile is left as it is
            unsigned old = __hip_atomic_load(q.inq + nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                const unsigned want = old == 0u ? 1u : old == 2u ? 3u : old;
                if (want == old) return;
                const unsigned got = atomicCAS(q.inq + nb, old, want);
                if (got == old) break;
                old = got;
            }
            if (old == 0u) enqueue(nb);
        };
        if constexpr (PLAIN)
            recon_tile_plain<CONN, true>(a, item, q.max_sweeps, lds, push);
        else
            recon_tile<T, CONN, true>(a, item, q.max_sweeps, reinterpret_cast<int (*)[65]>(lds), push);
        __syncthreads();
        if (lane == 0) {
            // leave the visit; pushed meanwhile (3): queue the tile again
            // (pushers leave state 3 alone, so the exchange below is safe)
            if (atomicCAS(q.inq + item, 2u, 0u) != 2u) {
                atomicExch(q.inq + item, 1u);
                enqueue(item);
            }
            atomicAdd(done, 1u);
            atomicSub(pending, 1u);
        }
    }
}

// Seeding from the worklist a round left behind (count on the device): the
// first kernel empties the ring and the in-queue flags, the second puts the
// listed tiles under tickets 0 .. count-1.
__global__ void k_queue_clear(QueueArgs q) {
    const int cap = 2 * q.total;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
        q.ring[i] = RING_EMPTY;
        if (i < q.total) q.inq[i] = 0u;
    }
}

__global__ void k_queue_seed(QueueArgs q, const int32_t *list, const int32_t *count) {
    const int nl = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
        const int tile = list[i];
        q.ring[i] = ((unsigned long long)i << 32) | (unsigned)tile;
        q.inq[tile] = 1u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        q.ctl[0] = 0u;
        q.ctl[1] = (unsigned)nl;
        q.ctl[2] = (unsigned)nl;
        q.ctl[3] = 0u;
        q.ctl[4] = 0u;
    }
}

__global__ void k_queue_init(QueueArgs q) {
    const int cap = 2 * q.total;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
        q.ring[i] = i < q.total ? (((unsigned long long)i << 32) | (unsigned)i) : RING_EMPTY;
        if (i < q.total) q.inq[i] = 1u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        q.ctl[0] = 0u;
        q.ctl[1] = (unsigned)q.total;
        q.ctl[2] = (unsigned)q.total;
        q.ctl[3] = 0u;
        q.ctl[4] = 0u;
    }
}

template <typename T, int CONN, bool QUEUE, typename Push>
__device__ void recon_tile(const ReconImg &a, int gtile, int max_sweeps, int (*Ts)[65], Push push) {
    const int lane = threadIdx.x;
    const int tile = gtile - a.unit0;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    // the register block covers the interior [x0, x0+62) x [y0, y0+62) and a
    // one-pixel ring: block coordinate (i, j) is image pixel (x0-1+i, y0-1+j)
    const int x0 = tx * RIN, y0 = ty * RIN;
    const T *mask = static_cast<const T *>(a.mask);
    T *rr = static_cast<T *>(a.r);

    int r[64];
    MaskRegs<T> mc, mr;
    mc.clear();
    mr.clear();
    const int gx = x0 - 1 + lane;
    const bool col_inner = lane >= 1 && lane <= 62;
    if (sizeof(T) == 1 && a.domain == nullptr) {
        // every load first (clamped addresses, no branch between them), so
        // that they are all in flight together; then the out-of-image values
        // become NEG
        const bool col_ok = gx >= 0 && gx < a.w;
        const int gxc = min(max(gx, 0), a.w - 1);
        // the images are in global memory: global loads from a uniform base
        // and a 32-bit offset instead of generic ones with 64-bit addresses
        typedef const __attribute__((address_space(1))) T *gptr;
        const gptr grr = (gptr)rr, gmask = (gptr)mask;
        T rv[64], mv[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            // uniform row start, per-lane 32-bit column
            const int64_t row = (int64_t)min(max(y0 - 1 + j, 0), a.h - 1) * a.pitch;
            rv[j] = (grr + row)[gxc];
            mv[j] = (gmask + row)[gxc];
        }
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const int gy = y0 - 1 + j;
            const bool ok = col_ok && gy >= 0 && gy < a.h;
            r[j] = ok ? (int)rv[j] : NEG;
            // ring pixels are read-only: they carry mask NEG
            const int m = (ok && col_inner && j >= 1 && j <= 62) ? (int)mv[j] : NEG;
            mc.set(j, m);
            Ts[j][lane] = m;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const int gy = y0 - 1 + j;
            r[j] = gval<T>(a, rr, gx, gy);
            // ring pixels are read-only: they carry mask NEG
            const int mv = (col_inner && j >= 1 && j <= 62) ? gval<T>(a, mask, gx, gy) : NEG;
            mc.set(j, mv);
            Ts[j][lane] = mv;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 64; ++i) mr.set(i, Ts[lane][i]);
    __syncthreads();
    // original interior edge values (row 1 / row 62 per lane = column,
    // column 1 / column 62 per lane = row, through the transpose below)
    const int oT = r[1], oB = r[62];
#pragma unroll
    for (int j = 0; j < 64; ++j) Ts[j][lane] = r[j];
    __syncthreads();
    const int oL = Ts[lane][1], oR = Ts[lane][62];
    __syncthreads();

    bool any_change = false;
    bool converged = false;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        bool ch = false;
        // down and up, lane = column; ring lanes never change and feed their
        // values to the DPP shifts like any other lane
        {
            int pc = r[0];
            int pl = shr0(pc), pr = shl0(pc);
#pragma unroll
            for (int j = 1; j < 64; ++j) {
                const int m = CONN == 8 ? max(pc, max(pl, pr)) : pc;
                const int nv = step_val(r[j], m, mc.eff(j));
                ch |= nv != r[j];
                r[j] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr0(nv);
                    pr = shl0(nv);
                }
            }
            pc = r[63];
            pl = shr0(pc);
            pr = shl0(pc);
#pragma unroll
            for (int j = 62; j >= 0; --j) {
                const int m = CONN == 8 ? max(pc, max(pl, pr)) : pc;
                const int nv = step_val(r[j], m, mc.eff(j));
                ch |= nv != r[j];
                r[j] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr0(nv);
                    pr = shl0(nv);
                }
            }
        }
        // transpose: lane = row
#pragma unroll
        for (int j = 0; j < 64; ++j) Ts[j][lane] = r[j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 64; ++i) r[i] = Ts[lane][i];
        __syncthreads();
        // right and left, lane = row
        {
            int pc = r[0];
            int pl = shr0(pc), pr = shl0(pc);
#pragma unroll
            for (int i = 1; i < 64; ++i) {
                const int m = CONN == 8 ? max(pc, max(pl, pr)) : pc;
                const int nv = step_val(r[i], m, mr.eff(i));
                ch |= nv != r[i];
                r[i] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr0(nv);
                    pr = shl0(nv);
                }
            }
            pc = r[63];
            pl = shr0(pc);
            pr = shl0(pc);
#pragma unroll
            for (int i = 62; i >= 0; --i) {
                const int m = CONN == 8 ? max(pc, max(pl, pr)) : pc;
                const int nv = step_val(r[i], m, mr.eff(i));
                ch |= nv != r[i];
                r[i] = nv;
                pc = nv;
                if (CONN == 8) {
                    pl = shr0(nv);
                    pr = shl0(nv);
                }
            }
        }
        // transpose back: lane = column (Ts keeps the row-major copy)
#pragma unroll
        for (int i = 0; i < 64; ++i) Ts[lane][i] = r[i];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 64; ++j) r[j] = Ts[j][lane];
        __syncthreads();
        if (!wave_any(ch)) {
            converged = true;
            break;
        }
        any_change = true;
    }
    if (!any_change) return;

    // write back the interior members (own column)
#pragma unroll
    for (int j = 1; j < 63; ++j) {
        const int gy = y0 - 1 + j;
        if (mc.eff(j) != NEG) rr[(int64_t)gy * a.pitch + gx] = (T)r[j];
    }
    // which interior edges changed?
    const bool cT = col_inner && r[1] != oT, cB = col_inner && r[62] != oB;
    const bool row_inner = lane >= 1 && lane <= 62;
    const bool cL = row_inner && Ts[lane][1] != oL, cR = row_inner && Ts[lane][62] != oR;
    const uint64_t mT = __ballot(cT), mB = __ballot(cB), mL = __ballot(cL), mR = __ballot(cR);
    if constexpr (QUEUE) __threadfence();   // release the tile's writes before announcing them
    // the list is the same in every lane; lane k pushes entry k
    int nb[9];
    int nn = 0;
    auto add = [&](int dx, int dy) {
        int nx = tx + dx, ny = ty + dy;
        if (nx >= 0 && ny >= 0 && nx < a.ntx && ny < a.nty) nb[nn++] = a.unit0 + ny * a.ntx + nx;
    };
    if (mT) add(0, -1);
    if (mB) add(0, 1);
    if (mL) add(-1, 0);
    if (mR) add(1, 0);
    if (CONN == 8) {
        if ((mT >> 1) & 1ull) add(-1, -1);   // interior corner (1, 1)
        if ((mT >> 62) & 1ull) add(1, -1);   // (62, 1)
        if ((mB >> 1) & 1ull) add(-1, 1);    // (1, 62)
        if ((mB >> 62) & 1ull) add(1, 1);    // (62, 62)
    }
    if (!converged) nb[nn++] = gtile;  // sweep budget exhausted: continue later
    int mine = -1;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (k == lane && k < nn) mine = nb[k];
    push(mine, lane < nn);
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

int recon_init(int dtype, const void *marker, const void *mask, void *out, int w, int h, int64_t pitch,
               hipStream_t s) {
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

__global__ void k_batch_begin(const BatchAux *aux, int n, int32_t *shared_ctr, int n_ctr) {
    const int i = blockIdx.x;
    if (i == n) {
        for (int k = threadIdx.x; k < n_ctr; k += blockDim.x) shared_ctr[k] = 0;
        return;
    }
    const BatchAux a = aux[i];
    for (int k = threadIdx.x; k < 256 * HIST_COPIES; k += blockDim.x) a.hist[k] = 0;
    if (threadIdx.x == 0) *a.kept = 0;
}

// Level choice for the connectivity lower bound: the bound helps most around
// the density at which the upper level set {v >= l} stops percolating (about
// 0.41 for 8-connected sites), so the n levels are the smallest values whose
// upper-set density drops to n targets spread over [0.33, 0.75].
//
// Band selection: v0 = the highest value with at least frac of the pixels at
// or above it, and the levels v0 - n + 2 .. v0 + 1 (n = 1: v0 alone).  The
// reconstruction of the frame marker under Hq is the largest value at which
// a pixel is still joined to the frame, so wherever the upper level sets of a
// noisy background stop spanning the tile, the result has one plateau that
// covers most of the background at the last spanning level; the level set
// at that value then holds about half of the pixels.  Levels at and just
// above that value make the bound exact on the plateau and on the thin
// clusters that stay joined to the frame one step higher, which otherwise
// take the longest propagation.
//
// Threshold levels of the connectivity bound from the Hq histogram, one wave
// per image: lane t owns bins 4t .. 4t+3 and the counts of pixels at or above
// each bin come from a suffix sum over the lanes.  Mode 1 (band): v0 is the
// highest value whose upper set holds at least frac_permille / 1000 of the
// pixels, and the levels are v0 - n + 2 .. v0 + 1.  Mode 0 (quantiles): level
// k is the lowest value whose upper set holds at most q_k of the pixels, q_k
// from 0.75 down to 0.33.  In both modes the levels are non-decreasing in k,
// which the writer of the bound relies on.
__global__ __launch_bounds__(64) void k_batch_levels(const BatchAux *aux, int n_levels, int mode, int frac_permille) {
    const BatchAux a = aux[blockIdx.x];
    const int t = threadIdx.x;
    // the histogram copies sit in the arena (256-byte aligned): 16-byte loads
    const uint4 *hv = reinterpret_cast<const uint4 *>(a.hist);
    uint32_t h[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < HIST_COPIES; ++c) {
        const uint4 q = hv[c * 64 + t];
        h[0] += q.x;
        h[1] += q.y;
        h[2] += q.z;
        h[3] += q.w;
    }
    const uint32_t mine = h[0] + h[1] + h[2] + h[3];
    // inclusive suffix sum over the lanes: lane t gets the pixels of bins >= 4t
    uint32_t suf = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_down(suf, d, 64);
        if (t + d < 64) suf += o;
    }
    const uint32_t total = __shfl(suf, 0, 64);
    uint32_t above[4];   // pixels with value >= 4t + j
    above[0] = suf;
#pragma unroll
    for (int j = 1; j < 4; ++j) above[j] = above[j - 1] - h[j - 1];
    if (mode == 1) {
        // v0: the highest value whose upper set holds at least frac of the pixels (0 if none)
        const double need = (double)total * frac_permille / 1000.0;
        int v0 = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((double)above[j] >= need) v0 = 4 * t + j;
        for (int d = 32; d > 0; d >>= 1) v0 = max(v0, __shfl_xor(v0, d, 64));
        if (t == 0) {
            const int top = n_levels == 1 ? v0 : min(v0 + 1, 255);
            for (int k = 0; k < n_levels; ++k) a.levels[k] = max(1, top - (n_levels - 1 - k));
        }
    } else {
        // level k: the lowest value whose upper set holds at most q_k of the
        // pixels, q_k from 0.75 down to 0.33 (255 if none)
        for (int k = 0; k < n_levels; ++k) {
            const double q = n_levels == 1 ? 0.5 : 0.75 - 0.42 * k / (n_levels - 1);
            int v = 256;
#pragma unroll
            for (int j = 3; j >= 0; --j)
                if ((double)above[j] <= q * (double)total) v = 4 * t + j;
            for (int d = 32; d > 0; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
            if (t == 0) a.levels[k] = v == 256 ? 255 : max(v, 1);
        }
    }
}

__global__ void k_batch_end(const BatchAux *aux, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && aux[i].n_dev) *aux[i].n_dev = *aux[i].kept;
}

// R0 = J: the frame marker (Hq on the 1-pixel tile frame, 0 inside); image =
// blockIdx.y
__global__ void k_batch_frame_marker(const BatchAux *aux) {
    const BatchAux a = aux[blockIdx.y];
    const int64_t n = (int64_t)a.w * a.h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / a.w, x = i - y * a.w;
        const bool fr = x == 0 || y == 0 || x == a.w - 1 || y == a.h - 1;
        a.R[i] = fr ? a.hq[i] : 0;
    }
}

// zeroes the optional foreground / seed maps of every image (image = blockIdx.y)
__global__ void k_batch_zero_maps(const BatchAux *aux) {
    const BatchAux a = aux[blockIdx.y];
    if (!a.fg_out) return;
    const int64_t n = (int64_t)a.w * a.h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / a.w, x = i - y * a.w;
        a.fg_out[y * a.out_pitch + x] = 0;
        a.seeds_out[y * a.out_pitch + x] = 0;
    }
}

int launch_batch_zero_maps(const BatchAux *aux, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_zero_maps, dim3(64, n), dim3(256), 0, s, aux);
    return hip_fail(hipGetLastError(), "k_batch_zero_maps");
}

int launch_batch_begin(const BatchAux *aux, int n, int32_t *shared_ctr, int n_ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_begin, dim3(n + 1), dim3(256), 0, s, aux, n, shared_ctr, n_ctr);
    return hip_fail(hipGetLastError(), "k_batch_begin");
}
int launch_batch_levels(const BatchAux *aux, int n, int n_levels, int mode, int frac_permille, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_levels, dim3(n), dim3(64), 0, s, aux, n_levels, mode, frac_permille);
    return hip_fail(hipGetLastError(), "k_batch_levels");
}
int launch_batch_frame_marker(const BatchAux *aux, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_frame_marker, dim3(256, n), dim3(256), 0, s, aux);
    return hip_fail(hipGetLastError(), "k_batch_frame_marker");
}
int launch_batch_end(const BatchAux *aux, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_end, dim3((n + 63) / 64), dim3(64), 0, s, aux, n);
    return hip_fail(hipGetLastError(), "k_batch_end");
}

// Start of a reconstruction: no tile stamped, the three list counters zero
// (one launch for both).
// Device-side finish of a reconstruction after the launched rounds (no host
// read of the worklist): one workgroup runs rounds k0, k0 + 1, ... itself,
// each over the list the previous round left, visiting its tiles one after
// the other, until a round starts with an empty list.  The rounds keep the
// launched rounds' lists, counters and stamps (round k reads counter k % 3,
// writes (k + 1) % 3, clears (k + 2) % 3); an agent-scope fence after every
// tile visit publishes its writes to the next visits, whose loads it orders.
// With enough launched rounds the list is already empty and the workgroup
// leaves at once.
template <typename T, int CONN, bool PLAIN>
__global__ __launch_bounds__(64) void k_recon_finisher(RoundArgs ra, int32_t *lists, int k0) {
    __shared__ __align__(16) uint8_t lds[PLAIN ? PLAIN_LDS : 64 * 65 * 4];
    const int lane = threadIdx.x;
    for (int k = k0;; ++k) {
        __threadfence();
        int32_t *cnt_in = ra.cnt + (k % 3), *cnt_out = ra.cnt + ((k + 1) % 3), *cnt_clr = ra.cnt + ((k + 2) % 3);
        const int n_in = __hip_atomic_load(cnt_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n_in == 0) break;
        if (lane == 0) __hip_atomic_store(cnt_clr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t *list_in = lists + (k & 1) * (size_t)ra.total;
        int32_t *list_out = lists + ((k + 1) & 1) * (size_t)ra.total;
        const uint32_t epoch = (uint32_t)k + 1;
        if (ra.visits && lane == 0) atomicAdd(ra.visits, (unsigned long long)n_in);
        for (int slot = 0; slot < n_in; ++slot) {
            const int gtile = list_in[slot];
            const ReconImg a = ra.imgs[recon_img_of(ra.imgs, ra.n, gtile)];
            auto push = [&](int item, bool valid) {
                const bool fresh = valid && atomicExch(ra.stamp + item, epoch) != epoch;
                const uint64_t m = __ballot(fresh);
                if (!m) return;
                int base = 0;
                if (lane == 0) base = atomicAdd(cnt_out, __popcll(m));
                base = __shfl(base, 0, 64);
                if (fresh) list_out[base + __popcll(m & ((1ull << lane) - 1))] = item;
            };
            if constexpr (PLAIN)
                recon_tile_plain<CONN, false>(a, gtile, ra.max_sweeps, lds, push);
            else
                recon_tile<T, CONN, false>(a, gtile, ra.max_sweeps, reinterpret_cast<int (*)[65]>(lds), push);
            __syncthreads();
            __threadfence();
        }
    }
}

__global__ void k_recon_reset(uint32_t *stamp, int total, int32_t *cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) stamp[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x < 3) cnt[threadIdx.x] = 0;
}

template <typename T, int CONN, bool PLAIN = false>
static void launch_round(const RoundArgs &ra, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_recon_round<T, CONN, PLAIN>), dim3(grid), dim3(64), 0, s, ra);
}

int64_t recon_tiles(int w, int h) { return (int64_t)((w + RIN - 1) / RIN) * ((h + RIN - 1) / RIN); }

int recon_prepare(rt_ctx_impl *c, int total, ReconRun &run) {
    int e = ensure_stamps(c, (size_t)total);
    if (e) return e;
    int32_t *lists = (int32_t *)c->arena.take(sizeof(int32_t) * (2 * (size_t)total + 4));
    if (!lists) {
        set_error("recon: scratch arena too small");
        return RT_ENOMEM;
    }
    run.lists = lists;
    run.cnt = lists + 2 * (size_t)total;
    run.total = total;
    run.ring = (unsigned long long *)c->arena.take(sizeof(unsigned long long) * 2 * (size_t)std::max(total, 1));
    run.qctl = (unsigned int *)c->arena.take(sizeof(unsigned int) * 8);
    run.inq = (unsigned int *)c->arena.take(sizeof(unsigned int) * (size_t)std::max(total, 1));
    if (!run.ring || !run.qctl || !run.inq) {
        set_error("recon: scratch arena too small");
        return RT_ENOMEM;
    }
    return RT_OK;
}

// Rounds k0 .. k1-1.  Round k reads list k & 1 (all tiles when k == 0) and
// counter k % 3, writes list (k+1) & 1 and counter (k+1) % 3, and clears
// counter (k+2) % 3.  A tile is queued once per round: its stamp holds the
// number of the round that queued it (k + 1); the stamps are cleared at k = 0.
int recon_launch(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn, int k0,
                 int k1, hipStream_t s) {
    RoundArgs ra;
    ra.imgs = imgs_dev;
    ra.n = n;
    ra.total = run.total;
    ra.cnt = run.cnt;
    ra.stamp = c->stamps;
    ra.max_sweeps = c->knobs.recon_max_sweeps;
    const int grid = std::min(run.total, c->n_cu * 8);
    if (run.total <= 0) return RT_OK;
    if (k0 == 0) {
        hipLaunchKernelGGL(k_recon_reset, dim3(std::min((run.total + 255) / 256, 1024)), dim3(256), 0, s, c->stamps,
                           run.total, run.cnt);
        RT_HIP(hipGetLastError());
    }
    ra.visits = c->prof_on ? c->prof_visits : nullptr;
    hipEvent_t ev_end = nullptr;
    if (c->prof_on && k1 > k0) {
        // timing of the round kernel: one pair of events around these
        // consecutive launches (the gaps between them count as kernel time)
        while (c->round_events.size() < c->round_used + 2) {
            hipEvent_t ev;
            RT_HIP(hipEventCreate(&ev));
            c->round_events.push_back(ev);
        }
        RT_HIP(hipEventRecord(c->round_events[c->round_used], s));
        ev_end = c->round_events[c->round_used + 1];
        c->round_used += 2;
        c->round_launches += k1 - k0;
    }
    for (int k = k0; k < k1; ++k) {
        ra.k = k;
        ra.first = k == 0;
        ra.list_in = run.lists + (k & 1) * (size_t)run.total;
        ra.list_out = run.lists + ((k + 1) & 1) * (size_t)run.total;
        ra.epoch = (uint32_t)k + 1;
        if (dtype == RECON_U8_PLAIN) {
            // two waves per SIMD fit the plain kernel's registers: a grid of
            // exactly the resident workgroups (larger grids measured slower:
            // workgroups that start late hold back the round's end)
            const int g = std::min(run.total, c->n_cu * 8);
            if (conn == 8) launch_round<uint8_t, 8, true>(ra, g, s);
            else launch_round<uint8_t, 4, true>(ra, g, s);
        } else if (dtype == RT_U8) {
            if (conn == 8) launch_round<uint8_t, 8>(ra, grid, s);
            else launch_round<uint8_t, 4>(ra, grid, s);
        } else {
            if (conn == 8) launch_round<int32_t, 8>(ra, grid, s);
            else launch_round<int32_t, 4>(ra, grid, s);
        }
        RT_HIP(hipGetLastError());
    }
    if (ev_end) RT_HIP(hipEventRecord(ev_end, s));
    return RT_OK;
}

int recon_finish_device(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn,
                        int k0, hipStream_t s) {
    if (run.total <= 0) return RT_OK;
    if (k0 < 1) {
        set_error("recon: the device finish follows at least one launched round");
        return RT_EINVAL;
    }
    RoundArgs ra{};
    ra.imgs = imgs_dev;
    ra.n = n;
    ra.total = run.total;
    ra.cnt = run.cnt;
    ra.stamp = c->stamps;
    ra.max_sweeps = c->knobs.recon_max_sweeps;
    ra.visits = c->prof_on ? c->prof_visits : nullptr;
    if (dtype == RECON_U8_PLAIN) {
        if (conn == 8) hipLaunchKernelGGL((k_recon_finisher<uint8_t, 8, true>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
        else hipLaunchKernelGGL((k_recon_finisher<uint8_t, 4, true>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
    } else if (dtype == RT_U8) {
        if (conn == 8) hipLaunchKernelGGL((k_recon_finisher<uint8_t, 8, false>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
        else hipLaunchKernelGGL((k_recon_finisher<uint8_t, 4, false>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
    } else {
        if (conn == 8) hipLaunchKernelGGL((k_recon_finisher<int32_t, 8, false>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
        else hipLaunchKernelGGL((k_recon_finisher<int32_t, 4, false>), dim3(1), dim3(64), 0, s, ra, run.lists, k0);
    }
    return hip_fail(hipGetLastError(), "k_recon_finisher");
}

int recon_queue(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn,
                hipStream_t s, int from_round) {
    if (run.total <= 0) return RT_OK;
    QueueArgs q;
    q.imgs = imgs_dev;
    q.n = n;
    q.total = run.total;
    q.ring = run.ring;
    q.ctl = run.qctl;
    q.inq = run.inq;
    q.max_sweeps = c->knobs.recon_max_sweeps;
    q.spin_limit = 200000;   // 2 ms at the 100 MHz wall clock
    q.visits = c->prof_on ? c->prof_visits : nullptr;
    const int gi = (int)std::min<int64_t>((2 * (int64_t)run.total + 255) / 256, 1024);
    if (from_round <= 0) {
        hipLaunchKernelGGL(k_queue_init, dim3(gi), dim3(256), 0, s, q);
    } else {
        // the list that round from_round - 1 wrote, counted by counter from_round % 3
        hipLaunchKernelGGL(k_queue_clear, dim3(gi), dim3(256), 0, s, q);
        RT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_queue_seed, dim3(gi), dim3(256), 0, s, q,
                           (const int32_t *)(run.lists + (from_round & 1) * (size_t)run.total),
                           (const int32_t *)(run.cnt + (from_round % 3)));
    }
    RT_HIP(hipGetLastError());
    hipEvent_t ev_end = nullptr;
    if (c->prof_on) {
        while (c->round_events.size() < c->round_used + 2) {
            hipEvent_t ev;
            RT_HIP(hipEventCreate(&ev));
            c->round_events.push_back(ev);
        }
        RT_HIP(hipEventRecord(c->round_events[c->round_used], s));
        ev_end = c->round_events[c->round_used + 1];
        c->round_used += 2;
        c->round_launches += 1;
    }
    // every wave resident: 2 waves per SIMD fit the kernel's registers
    const int grid = std::min(run.total, c->n_cu * 8);
    if (dtype == RECON_U8_PLAIN) {
        if (conn == 8) hipLaunchKernelGGL((k_recon_queue<uint8_t, 8, true>), dim3(grid), dim3(64), 0, s, q);
        else hipLaunchKernelGGL((k_recon_queue<uint8_t, 4, true>), dim3(grid), dim3(64), 0, s, q);
    } else if (dtype == RT_U8) {
        if (conn == 8) hipLaunchKernelGGL((k_recon_queue<uint8_t, 8, false>), dim3(grid), dim3(64), 0, s, q);
        else hipLaunchKernelGGL((k_recon_queue<uint8_t, 4, false>), dim3(grid), dim3(64), 0, s, q);
    } else {
        if (conn == 8) hipLaunchKernelGGL((k_recon_queue<int32_t, 8, false>), dim3(grid), dim3(64), 0, s, q);
        else hipLaunchKernelGGL((k_recon_queue<int32_t, 4, false>), dim3(grid), dim3(64), 0, s, q);
    }
    RT_HIP(hipGetLastError());
    if (ev_end) RT_HIP(hipEventRecord(ev_end, s));
    return RT_OK;
}

int recon_queue_aborted(rt_ctx_impl *c, const ReconRun &run, hipStream_t s, int *aborted) {
    *aborted = 0;
    if (run.total <= 0) return RT_OK;
    RT_HIP(hipMemcpyAsync(c->pinned, run.qctl + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    c->recon_host_reads++;
    *aborted = c->pinned[0] != 0;
    return RT_OK;
}

int recon_pending(rt_ctx_impl *c, const ReconRun &run, int k, hipStream_t s, int *pending) {
    if (run.total <= 0) {
        *pending = 0;
        return RT_OK;
    }
    // the list produced by round k-1 is counted by counter k % 3
    RT_HIP(hipMemcpyAsync(c->pinned, run.cnt + (k % 3), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    c->recon_host_reads++;
    *pending = c->pinned[0];
    return RT_OK;
}

int recon_finish(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn, int k0,
                 hipStream_t s, int *rounds_out) {
    const int batch = c->knobs.recon_round_batch;
    const int max_rounds = 1 << 20;
    int k = k0;
    for (;;) {
        if (k > 0) {
            int pending = 0;
            int e = recon_pending(c, run, k, s, &pending);
            if (e) return e;
            if (!pending) break;
        }
        if (k > max_rounds) {
            set_error("recon: no convergence after %d rounds", k);
            return RT_EDEVICE;
        }
        int e = recon_launch(c, run, imgs_dev, n, dtype, conn, k, k + batch, s);
        if (e) return e;
        k += batch;
    }
    if (rounds_out) *rounds_out = k;
    return RT_OK;
}

int recon_rounds(rt_ctx_impl *c, const ReconImg *imgs_dev, int n, int dtype, int conn, int total, hipStream_t s,
                 int *rounds_out) {
    const size_t mark = c->arena.off;
    ReconRun run;
    int e = recon_prepare(c, total, run);
    if (!e && c->knobs.recon_mode != 0) {
        int aborted = 0;
        const int kq = c->knobs.recon_mode == 2 ? c->knobs.recon_queue_after : 0;
        if (kq > 0) e = recon_launch(c, run, imgs_dev, n, dtype, conn, 0, kq, s);
        if (!e) e = recon_queue(c, run, imgs_dev, n, dtype, conn, s, kq);
        if (!e) e = recon_queue_aborted(c, run, s, &aborted);
        if (!e && aborted) e = recon_finish(c, run, imgs_dev, n, dtype, conn, 0, s, rounds_out);
        else if (rounds_out) *rounds_out = kq + 1;
    } else if (!e) {
        e = recon_finish(c, run, imgs_dev, n, dtype, conn, 0, s, rounds_out);
    }
    c->arena.off = mark;
    return e;
}

}  // namespace rtseg
