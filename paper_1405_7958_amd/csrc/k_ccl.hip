// Connected-component labelling by union-find (BWLabel, Sec. 5.1: a forest
// in which every pixel starts as its own tree, adjacent trees are merged, and
// labels are read off by flattening the trees).
//
// One wavefront per 64 x 64 tile.  A row of the tile is one 64-bit mask, so
// the forest is built over horizontal runs instead of pixels: the pixels of a
// run share its first pixel as parent by construction (bit arithmetic, no
// atomics), and only runs of adjacent rows that touch are united (LDS
// atomicMin, the root is always the smallest index, so labels are canonical
// by construction).  Two run starts of one row are at least two pixels apart,
// so the forest needs one LDS slot per pixel pair.  Three launches:
//   local  : build the tile forest; publish its border-touching roots to
//            the global id array (id 0 = virtual node, pixel p has id p + 1)
//            and, in the tile's border table, each border pixel's local
//            root (or -1);
//   merge  : one wave per tile edge unites, across the tile's right or
//            bottom edge, each pair of touching edge runs once (global
//            atomicMin), starting from the local roots in the two tables;
//   flatten: BWLabel rebuilds the tile forest (it costs 1 byte/pixel of
//            input instead of 4 bytes/pixel of stored local roots), finds
//            each local root's global root once, and writes the labels;
//            FillHoles and the bound look up only the border runs' roots
//            (from the border table) and flood the frame-connected set inside
//            the tile.
// Modes: BWLabel (labels, per-component area and bounding box, component
// list), FillHoles (background components joined to a virtual frame node),
// and the multi-level frame-connectivity lower bound that starts the
// grayscale reconstruction.  In the multi-level mode the local phase takes
// one wave per (tile, level) and the merge one wave per (level, edge) of a
// tile, so the levels' forests and global unions proceed side by side; the
// flatten holds one wave per level of a tile in a workgroup and combines the
// levels' frame-connected pixel sets in LDS before one write of the bound.
//
// Every kernel is specialised for its predicate and output, so each one is
// straight-line code for its own mode.  Tile rows are read with 16-byte loads
// (four per lane cover the tile) and turned into row masks lane-locally.
#include "rt_internal.h"

namespace rtseg {

constexpr int CT = 64;                 // tile edge = wavefront size
constexpr int MAXLEV = 8;
constexpr int NSLOT = CT * CT / 2;     // forest slots: one per pixel pair of a row
constexpr int FRAME_BIT = 1 << 12;     // tags a local root whose component touches the image frame
constexpr int TOUCH_BIT = 1 << 13;     // tags a local root whose component touches the tile border
constexpr int LIDX = 0xfff;
constexpr int NLIST = 128;             // components touching a tile border: at most 126 (one per two border pixels)
constexpr int NHASH = 64;              // per-tile component table of the statistics pass
// After the row masks and the 32-bit forest, one region holds first the root
// list of the global lookups and then the statistics table (key, area with
// the root flag, x0, x1, y0, y1): 10,240 bytes per BWLabel tile, so that 16
// tiles share a CU's 160 KB.
constexpr int TAIL_LDS = NHASH * 6 * 4;
static_assert(TAIL_LDS >= NLIST * 4 + 4, "the root list and its count fit the table's space");
constexpr int WAVE_LDS = CT * 8 + NSLOT * 4 + TAIL_LDS;
constexpr int LABELS_LDS = WAVE_LDS;
constexpr int ROOT_FLAG = 1 << 30;     // statistics table area: the component's root run lies in this tile
constexpr int LOCAL_LDS = CT * 8 + NSLOT * 2;   // local phase: row masks + 16-bit forest

extern __shared__ uint64_t ccl_smem[];

__device__ __forceinline__ int lane_id() { return threadIdx.x & (CT - 1); }

struct WaveMem {
    uint64_t *rows;   // rows[y] bit x = member (x, y)
    int *P;           // forest over run starts, indexed by slot()
    int *list;        // border-touching roots of the tile (then the statistics table)
    int *count;       // their number
};

__device__ __forceinline__ WaveMem wave_mem(int wave) {
    uint64_t *base = ccl_smem + (size_t)wave * (WAVE_LDS / 8);
    int *P = (int *)(base + CT);
    return {base, P, P + NSLOT, P + NSLOT + NLIST};
}

// forest slot of the run start at tile index li = y * 64 + s: y * 32 + s / 2
// (one slot per pixel pair of a row), which is li / 2
__device__ __forceinline__ int slot(int li) { return li >> 1; }

// Forest entries: the tile index of the parent run start (12 bits) and the
// two tags.  The local phase keeps them in 16 bits (4 KB per tile, which
// doubles the waves an LDS budget holds); the BWLabel flatten keeps 32 bits,
// because it replaces the roots' entries by global ids.  A link at a root is
// an atomic minimum (for 16-bit entries a compare-and-swap of the 32-bit word
// that holds two of them); path halving may use plain stores, because a
// non-root entry only ever moves to another ancestor.
__device__ __forceinline__ int p_load(const int *P, int i) {
    return __hip_atomic_load(P + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void p_halve(int *P, int i, int v) { atomicMin(P + i, v); }
__device__ __forceinline__ int p_link(int *P, int i, int v) { return atomicMin(P + i, v); }
__device__ __forceinline__ void p_or(int *P, int i, int bits) { atomicOr(P + i, bits); }

__device__ __forceinline__ int p_load(const uint16_t *P, int i) {
    return __hip_atomic_load(P + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void p_halve(uint16_t *P, int i, int v) {
    __hip_atomic_store(P + i, (uint16_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int p_link(uint16_t *P, int i, int v) {   // atomic min, returns the old entry
    uint32_t *w = (uint32_t *)P + (i >> 1);
    const int sh = (i & 1) * 16;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const int cur = (int)((old >> sh) & 0xffffu);
        if (cur <= v) return cur;
        const uint32_t nw = (old & ~(0xffffu << sh)) | ((uint32_t)v << sh);
        const uint32_t got = atomicCAS(w, old, nw);
        if (got == old) return cur;
        old = got;
    }
}
__device__ __forceinline__ void p_or(uint16_t *P, int i, int bits) {
    atomicOr((uint32_t *)P + (i >> 1), (uint32_t)bits << ((i & 1) * 16));
}

// Finds with path halving: a node is re-pointed to its grandparent, so
// parent pointers only ever move to an ancestor and a concurrent link can
// never be undone.  Nodes are tile indices of run starts.
template <typename PT>
__device__ __forceinline__ int lfind(PT *P, int x) {
    int p = p_load(P, slot(x));
    while (p != x) {
        const int gp = p_load(P, slot(p));
        if (gp != p) p_halve(P, slot(x), gp);
        x = p;
        p = gp;
    }
    return x;
}

template <typename PT>
__device__ __forceinline__ void lunite(PT *P, int a, int b) {
    for (;;) {
        a = lfind(P, a);
        b = lfind(P, b);
        if (a == b) return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        const int old = p_link(P, slot(a), b);
        if (old == a) return;
        a = old;
    }
}

// Read-only find for the flatten pass: the forest no longer changes once the
// merge kernel has finished, so plain loads suffice and no path is rewritten
// (rewriting with atomics made every tile of a frame-spanning component
// contend on the same few nodes).
__device__ __forceinline__ int gfind_ro(const int32_t *ids, int x) {
    int p = ids[x];
    while (p != x) {
        x = p;
        p = ids[x];
    }
    return x;
}

// Both finds of a union walk their chains in the same loop, so that their
// dependent loads overlap (path halving on each, as gfind).
// Up to four read-only finds walked together (x[k] < 0: unused).  On
// return x[k] holds the root.
__device__ __forceinline__ void gfind4_ro(const int32_t *ids, int x[4]) {
    bool act[4];
    int q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        act[k] = x[k] >= 0;
        q[k] = act[k] ? ids[x[k]] : 0;
    }
    for (;;) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!act[k]) continue;
            if (q[k] == x[k]) {
                act[k] = false;
            } else {
                x[k] = q[k];
                any = true;
            }
        }
        if (!any) return;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (act[k]) q[k] = ids[x[k]];
    }
}

// The walks read the forest with plain loads, through the XCD's own L2, which
// may hold an older copy of a line that another XCD's atomics have changed
// since.  That is safe: parent links only ever move to smaller ancestors in
// the same set, so an older link is still a valid path to an ancestor (the
// walk ends, at a node that is or was a root), equal stale roots prove the two
// nodes joined, and linking is a device-scope atomic minimum that returns the
// true entry -- when the node is no longer a root the loop goes on from that
// entry, which is smaller each time.  Agent-scope loads would fetch a line
// from memory for every 4-byte node.
__device__ __forceinline__ void gunite(int32_t *ids, int a, int b) {
    for (;;) {
        int pa = ids[a], pb = ids[b];
        while (pa != a || pb != b) {
            const int ga = pa != a ? ids[pa] : a;
            const int gb = pb != b ? ids[pb] : b;
            if (pa != a) {
                if (ga != pa) atomicMin(ids + a, ga);
                a = pa;
                pa = ga;
            }
            if (pb != b) {
                if (gb != pb) atomicMin(ids + b, gb);
                b = pb;
                pb = gb;
            }
        }
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

// ---- 64-bit run arithmetic -------------------------------------------------
__device__ __forceinline__ uint64_t run_starts(uint64_t m) { return m & ~(m << 1); }
__device__ __forceinline__ int run_len(uint64_t m, int s) {   // m has bit s set
    uint64_t z = ~(m >> s);
    return z ? __builtin_ctzll(z) : 64 - s;
}
__device__ __forceinline__ int run_start_of(uint64_t m, int b) {   // m has bit b set
    uint64_t z = ~m & ((1ull << b) - 1);
    return z ? 64 - __builtin_clzll(z) : 0;
}

// The runs of m that hold a bit of s (s within m): adding s to m clears each
// run from its lowest seed to its end (the carry stops at the first zero);
// the same on the bit-reversed masks covers each run from its start to its
// highest seed.
__device__ __forceinline__ uint64_t run_fill(uint64_t m, uint64_t s) {
    s &= m;
    const uint64_t up = (m & ~(m + s)) | s;
    const uint64_t mr = __builtin_bitreverse64(m), sr = __builtin_bitreverse64(s);
    return up | __builtin_bitreverse64((mr & ~(mr + sr)) | sr);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Grows f (lane = row, within the row masks m) to everything connected to it
// inside the tile: each step takes the neighbour rows' pixels (and their
// diagonal neighbours for 8-connectivity) and fills whole runs, until no row
// changes.  The set only grows, so the loop ends.
__device__ uint64_t flood_rows(uint64_t m, uint64_t f, int conn) {
    const int lane = lane_id();
    f = run_fill(m, f);
    for (;;) {
        const uint64_t a = shfl64(f, lane > 0 ? lane - 1 : 0);
        const uint64_t b = shfl64(f, lane < CT - 1 ? lane + 1 : CT - 1);
        uint64_t nb = (lane > 0 ? a : 0ull) | (lane < CT - 1 ? b : 0ull);
        if (conn == 8) nb |= (nb << 1) | (nb >> 1);
        const uint64_t g = run_fill(m, f | nb);
        const bool grew = g != f;
        f = g;
        if (!__any(grew)) return f;
    }
}

// ---- predicate --------------------------------------------------------------
template <CclPred PR>
__device__ __forceinline__ bool pred_val(const CclArgs &A, uint32_t a, uint32_t b, int level) {
    if constexpr (PR == CclPred::NonZero) return a != 0;
    else if constexpr (PR == CclPred::Zero) return a == 0;
    else if constexpr (PR == CclPred::TophatBg) return (int)a - (int)b < A.t;
    else return (int)a >= level;
}


struct Tile {
    int tx, ty, x0, y0, tw, th;
};

__device__ __forceinline__ int img_of(const CclArgs *args, int n, int u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (args[mid].unit0 <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ Tile tile_of(const CclArgs &A, int b) {
    const int ntx = (A.w + CT - 1) / CT;
    Tile t;
    t.tx = b % ntx;
    t.ty = b / ntx;
    t.x0 = t.tx * CT;
    t.y0 = t.ty * CT;
    t.tw = min(CT, A.w - t.x0);
    t.th = min(CT, A.h - t.y0);
    return t;
}

__device__ __forceinline__ int gid(const CclArgs &A, const Tile &t, int x, int y) {
    return (t.y0 + y) * A.w + t.x0 + x + 1;
}

// Border table of tile b at level lev: 256 ints, the left column (index =
// row), the right column, the top row (index = column) and the bottom row;
// each entry is the id of the pixel's local root, or -1 for a non-member.
__device__ __forceinline__ int32_t *border_table(const CclArgs &A, int lev, int b) {
    const int64_t nt = (int64_t)((A.w + CT - 1) / CT) * ((A.h + CT - 1) / CT);
    return A.bt + (lev * nt + b) * 256;
}

__device__ __forceinline__ bool aligned16(const void *p, int64_t pitch) {
    return (((uintptr_t)p | (uintptr_t)pitch) & 15) == 0;
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &q, int i) {
    const uint32_t w = i < 4 ? q.x : i < 8 ? q.y : i < 12 ? q.z : q.w;
    return (w >> ((i & 3) * 8)) & 255u;
}

// The low 4 bits of x as the bytes of a word (bit k -> byte k, 0 or 1): the
// multiplier places bit k at bit 8k, and no two partial products overlap.
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t x) { return (__umul24(x & 15u, 0x204081u)) & 0x01010101u; }

// Loads the 16 bytes at p (nvalid of them inside the image; the rest read 0).
__device__ __forceinline__ uint4 load16(const uint8_t *p, int nvalid, bool wide) {
    if (wide && nvalid == 16) return *(const uint4 *)p;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int i = 0; i < nvalid; ++i) w[i >> 2] |= (uint32_t)p[i] << ((i & 3) * 8);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// rows[y] = member mask of tile row y.  Lane l reads rows l/4 + 16k (k < 4),
// columns 16 (l % 4) .. +15, and writes those 16 bits of the row mask.
template <CclPred PR>
__device__ void build_rows(const CclArgs &A, const Tile &t, int level, uint64_t *rows) {
    const int ln = lane_id();
    const int c = ln & 3;
    const int nvalid = max(0, min(16, t.tw - 16 * c));
    const bool wide_a = aligned16(A.a, A.pitch_a);
    const bool wide_b = PR == CclPred::TophatBg && aligned16(A.b, A.pitch_b);
    uint4 qa[4], qb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int y = (ln >> 2) + 16 * k;
        const int nv = y < t.th ? nvalid : 0;
        const int64_t gy = t.y0 + y;
        const int gx = t.x0 + 16 * c;
        qa[k] = load16(A.a + gy * A.pitch_a + gx, nv, wide_a);
        if constexpr (PR == CclPred::TophatBg) qb[k] = load16(A.b + gy * A.pitch_b + gx, nv, wide_b);
        else qb[k] = make_uint4(0, 0, 0, 0);
    }
    uint16_t *r16 = (uint16_t *)rows;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int y = (ln >> 2) + 16 * k;
        const int nv = y < t.th ? nvalid : 0;
        uint32_t bits = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) bits |= (pred_val<PR>(A, byte_of(qa[k], i), byte_of(qb[k], i), level) ? 1u : 0u) << i;
        bits &= (1u << nv) - 1u;
        r16[y * 4 + c] = (uint16_t)bits;
    }
    __syncthreads();
}

// The pixels of mask m's run that starts at bit s (adding that bit to m
// carries through the run and clears it), widened by one pixel on each side
// for 8-connectivity: the window in which a run of the row above touches it.
__device__ __forceinline__ uint64_t touch_window(uint64_t m, uint64_t bit, int conn) {
    const uint64_t run = m & ~(m + bit);
    return conn == 8 ? run | (run << 1) | (run >> 1) : run;
}

// Tile forest over runs.  Lane = row.  With FLAT, after the call
// P[slot(y*64+s)] = local root (tile index of a run start) for every run
// start s of row y; without it the forest is final but not flattened (a root
// is still its own entry, and lroot walks to it), which is all the local
// phase needs: it looks up the roots of border runs only.
//
// Built in three passes, so that no lane walks long parent chains:
//   1. every run takes as parent the first run of the row above that touches
//      it (plain stores, no finds);
//   2. pointer jumping re-points every run whose parent is not a root to its
//      grandparent, until all point at roots (the trees are at most 64 rows
//      deep, so at most six rounds; a run whose parent is a root stays done,
//      since no link happens in this pass; four runs of a lane per step keep
//      their loads in flight);
//   3. the runs that touch further runs above unite with them by union-find
//      (path halving, atomic links), on the now shallow forest.
// Parents always have smaller indices and links join roots by minimum, so
// the root of a component is its smallest run start, as with plain unions.
// Every pass is lane-divergent over the runs of a row, so each run's step is
// kept to a few 64-bit mask operations.
template <typename PT, bool FLAT = true>
__device__ void run_forest(const uint64_t *rows, PT *P, int conn) {
    const int y = lane_id();
    const int yb = y * CT;
    const uint64_t m = rows[y];
    const uint64_t pm = y > 0 ? rows[y - 1] : 0ull;
    const uint64_t ps = run_starts(pm);
    uint64_t more = 0;   // runs of row y that touch two or more runs above
    uint64_t pend = 0;   // runs of row y whose parent may not be a root
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const uint64_t bit = st & (0ull - st);
        const int s = __builtin_ctzll(st);
        const uint64_t w = touch_window(m, bit, conn);
        const uint64_t tm = pm & w;
        int par = yb + s;
        if (tm) {
            // the first touching run above: its start is the first touching
            // pixel, unless that run began left of the window; any other run
            // start in the window is a further touching run
            const int f = __builtin_ctzll(tm);
            const uint64_t wps = ps & w;
            int s2 = f;
            bool two;
            if ((ps >> f) & 1ull) {
                two = (wps & (wps - 1)) != 0;
            } else {
                s2 = run_start_of(pm, f);
                two = wps != 0;
            }
            par = yb - CT + s2;
            pend |= bit;
            if (two) more |= bit;
        }
        P[slot(yb + s)] = (PT)par;
    }
    __syncthreads();
    while (__any(pend != 0)) {
        uint64_t next = 0;
        for (uint64_t st = pend; st;) {
            // up to four runs; an empty place repeats the first run, so that
            // all loads are unconditional and in flight together
            int li[4], p[4], g[4];
            uint64_t bk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                bk[k] = st & (0ull - st);
                li[k] = st ? yb + __builtin_ctzll(st) : li[0];
                st ^= bk[k];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) p[k] = p_load(P, slot(li[k]));
#pragma unroll
            for (int k = 0; k < 4; ++k) g[k] = p_load(P, slot(p[k]));
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (bk[k] && g[k] != p[k]) {
                    p_halve(P, slot(li[k]), g[k]);
                    next |= bk[k];
                }
        }
        pend = next;
        __syncthreads();
    }
    for (uint64_t st = more; st; st &= st - 1) {
        const uint64_t bit = st & (0ull - st);
        const int s = __builtin_ctzll(st);
        const uint64_t w = touch_window(m, bit, conn);
        // the run starts in the window after the first touching pixel: the
        // touching runs other than the tree parent
        const uint64_t tm = pm & w;
        for (uint64_t o = ps & w & ~(tm & (0ull - tm)); o; o &= o - 1)
            lunite(P, yb + s, yb - CT + __builtin_ctzll(o));
    }
    __syncthreads();
    if constexpr (FLAT) {
        for (uint64_t st = run_starts(m); st; st &= st - 1) {
            const int li = yb + __builtin_ctzll(st);
            P[slot(li)] = (PT)lfind(P, li);
        }
        __syncthreads();
    }
}

// Root of run start x in a final forest, read-only; roots may carry tags.
template <typename PT>
__device__ __forceinline__ int lroot(const PT *P, int x) {
    int p = p_load(P, slot(x)) & LIDX;
    while (p != x) {
        x = p;
        p = p_load(P, slot(x)) & LIDX;
    }
    return x;
}

template <typename PT>
__device__ __forceinline__ int root_of(const uint64_t *rows, const PT *P, int x, int y) {
    return lroot(P, y * CT + run_start_of(rows[y], x));
}

// Tags the roots of components that reach the tile border.  Only those can
// be joined to other tiles; a component that touches the image frame touches
// the tile border too.  Lane = row.
template <typename PT>
__device__ void mark_touch(const Tile &t, const uint64_t *rows, PT *P) {
    const int lane = lane_id();
    // left and right columns (lane = row)
    if (lane < t.th) {
        const uint64_t m = rows[lane];
        if (m & 1ull) p_or(P, slot(root_of(rows, P, 0, lane)), TOUCH_BIT);
        if ((m >> (t.tw - 1)) & 1ull) p_or(P, slot(root_of(rows, P, t.tw - 1, lane)), TOUCH_BIT);
    }
    // top and bottom rows (lane = column): every run, at its start
    const int yb = t.th - 1;
    if ((run_starts(rows[0]) >> lane) & 1ull) p_or(P, slot(lroot(P, lane)), TOUCH_BIT);
    if (yb > 0 && ((run_starts(rows[yb]) >> lane) & 1ull)) p_or(P, slot(lroot(P, yb * CT + lane)), TOUCH_BIT);
    __syncthreads();
}

// The wave's threshold level in the multi-level mode (idle waves: an empty
// set, level 256).
template <CclPred PR>
__device__ __forceinline__ int wave_level(const CclArgs &A, int wave) {
    if constexpr (PR == CclPred::Level) return wave < A.n_levels ? A.levels[wave] : 256;
    else return 0;
}

// ---------------------------------------------------------------------------
// local phase
// ---------------------------------------------------------------------------
template <CclPred PR, CclOut OU>
__device__ __forceinline__ void ccl_local_tile(const CclArgs &A, int b, int wave) {
    const Tile t = tile_of(A, b);
    const int lane = lane_id();
    const bool live = PR != CclPred::Level || wave < A.n_levels;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    int32_t *ids = A.ids + (live ? wave : 0) * nid;
    if (live && b == 0 && lane == 0) ids[0] = 0;   // the virtual node is its own root
    uint64_t *rows = ccl_smem;
    uint16_t *P = (uint16_t *)(ccl_smem + CT);
    build_rows<PR>(A, t, wave_level<PR>(A, wave), rows);
    // the level sets hold many small components (short chains to walk), the
    // other sets few large ones, where one flattening pass beats long walks
    run_forest<uint16_t, PR != CclPred::Level>(rows, P, A.conn);
    // Roots of this lane's four border pixels (-1: not a member): column 0
    // and column tw - 1 of row `lane`, row 0 and row th - 1 of column `lane`.
    // The forest no longer changes (tags only go to root entries, and lroot
    // masks them), so every use below shares these.
    const int y = lane;
    const uint64_t m = rows[y];
    const int xr = t.tw - 1, yl = t.th - 1;
    const uint64_t top = rows[0], bot = rows[yl];
    const int r_l = (m & 1ull) ? lroot(P, y * CT) : -1;
    const int r_r = ((m >> xr) & 1ull) ? lroot(P, y * CT + run_start_of(m, xr)) : -1;
    const int r_t = ((top >> lane) & 1ull) ? lroot(P, run_start_of(top, lane)) : -1;
    const int r_b = ((bot >> lane) & 1ull) ? lroot(P, yl * CT + run_start_of(bot, lane)) : -1;
    const bool s_t = (run_starts(top) >> lane) & 1ull;   // a run of row 0 starts at column `lane`
    const bool s_b = (run_starts(bot) >> lane) & 1ull;   // the same for row th - 1
    // Tag the roots of components that reach the tile border (only those can
    // join other tiles) and, with a virtual frame node, of those that reach
    // the image frame (they reach the tile border too).  Rows are tagged once
    // per run, at its start.
    {
        const bool fv = A.frame_virtual;
        const int fl = fv && t.x0 == 0 ? FRAME_BIT : 0;
        const int fr = fv && t.x0 + t.tw == A.w ? FRAME_BIT : 0;
        const int ft = fv && t.y0 == 0 ? FRAME_BIT : 0;
        const int fb = fv && t.y0 + t.th == A.h ? FRAME_BIT : 0;
        if (r_l >= 0) p_or(P, slot(r_l), TOUCH_BIT | fl);
        if (r_r >= 0) p_or(P, slot(r_r), TOUCH_BIT | fr);
        if (s_t) p_or(P, slot(r_t), TOUCH_BIT | ft);
        if (s_b) p_or(P, slot(r_b), TOUCH_BIT | fb);
        __syncthreads();
    }
    if (!live) return;
    if constexpr (OU == CclOut::Labels) {
        // roots (lane = row): publish the touching ones, reset the statistics of all
        for (uint64_t st = run_starts(m); st; st &= st - 1) {
            const int s = __builtin_ctzll(st);
            const int li = y * CT + s;
            const int pv = P[slot(li)];
            if ((pv & LIDX) != li) continue;
            const int id = gid(A, t, s, y);
            if (pv & TOUCH_BIT) ids[id] = (pv & FRAME_BIT) ? 0 : id;
            if (A.st_area) {
                A.st_area[id] = 0;
                A.st_x0[id] = 0x7fffffff;
                A.st_y0[id] = 0x7fffffff;
                A.st_x1[id] = -1;
                A.st_y1[id] = -1;
            }
        }
    } else {
        // only the touching roots matter, and each is the root of a border
        // run: publish them from the border runs (the same value may be
        // written more than once)
        auto publish = [&](int r) {
            const int id = gid(A, t, r & (CT - 1), r >> 6);
            ids[id] = (p_load(P, slot(r)) & FRAME_BIT) ? 0 : id;
        };
        if (r_l >= 0) publish(r_l);
        if (r_r >= 0) publish(r_r);
        if (s_t) publish(r_t);
        if (yl > 0 && s_b) publish(r_b);
    }
    // the border table: the local root's id of each border pixel (-1: not a
    // member), four coalesced rows of 64
    int32_t *bt = border_table(A, live ? wave : 0, b);
    auto rid = [&](int r) { return r >= 0 ? gid(A, t, r & 63, r >> 6) : -1; };
    bt[lane] = rid(r_l);
    bt[64 + lane] = rid(r_r);
    bt[128 + lane] = rid(r_t);
    bt[192 + lane] = rid(r_b);
}

// One wave per (tile, level): unit u is tile u / nw at level u % nw.  The
// level sets' launch has 32 waves per CU, all resident only with at most 64
// registers a lane.
template <CclPred PR, CclOut OU>
__global__ __launch_bounds__(CT) __attribute__((amdgpu_waves_per_eu(PR == CclPred::Level ? 8 : 1))) void k_ccl_local(const CclArgs *args, int n, int total, int nw) {
    for (int u = blockIdx.x; u < total * nw; u += gridDim.x) {
        const int tu = u / nw;
        const CclArgs A = args[img_of(args, n, tu)];
        ccl_local_tile<PR, OU>(A, tu - A.unit0, u - tu * nw);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// merge phase: one wave per tile (and level), its right and bottom edges
// ---------------------------------------------------------------------------
// unites the pairs (a(i), b(i+d)), d in {-1,0,1} (8-conn) or {0} (4-conn),
// along an edge; a/b bit i = member at position i (b has two extra members
// at i = -1 and i = 64, passed as bm1 / b64; they lie in the diagonal
// neighbour tiles).  The nodes are the local roots of the edge pixels, from
// the border tables: ida = a(i)'s, idb_m / idb_0 / idb_p = those of b(i-1),
// b(i), b(i+1).  About one union per pair of touching runs: a pair is
// skipped when a pair with a lower position, together with an adjacency
// inside one tile (always joined by that tile's forest), implies it.
__device__ void edge_unions(int32_t *ids, uint64_t am, uint64_t bm, bool bm1, bool b64, int conn, int i, int ida,
                            int idb_m, int idb_0, int idb_p) {
    if (!((am >> i) & 1ull)) return;
    auto bset = [&](int j) -> bool {
        if (j == -1) return bm1;
        if (j == 64) return b64;
        if (j < -1 || j > 64) return false;
        return (bm >> j) & 1ull;
    };
    auto aset = [&](int j) -> bool { return j >= 0 && j < 64 && ((am >> j) & 1ull); };
    if (conn == 4) {
        if (!bset(i)) return;
        if (aset(i - 1) && bset(i - 1)) return;
        gunite(ids, ida, idb_0);
        return;
    }
    for (int d = -1; d <= 1; ++d) {
        int j = i + d;
        if (!bset(j)) continue;
        // implied by a(i-1) (same tile as a(i)) united with b(j)
        if (aset(i - 1) && j - (i - 1) <= 1 && j - (i - 1) >= -1) continue;
        // implied by a(i) united with b(j-1), when b(j-1) and b(j) lie in the
        // same tile (positions 0..63); across a tile corner the two edges
        // could otherwise each rely on the other's skipped union
        if (j >= 1 && j <= 63 && bset(j - 1) && (j - 1) - i <= 1 && (j - 1) - i >= -1) continue;
        gunite(ids, ida, d < 0 ? idb_m : d == 0 ? idb_0 : idb_p);
    }
}

// Wave 2l handles the right edge and wave 2l + 1 the bottom edge of the
// tile at level l, so the two edges' unions overlap.  Membership and the
// nodes come from the border tables the local phase wrote (coalesced rows,
// where the image's columns would be one cache line per pixel), and every
// union starts at a local root.
template <CclPred PR>
__device__ __forceinline__ void ccl_merge_tile(const CclArgs &A, int b, int wave) {
    const Tile t = tile_of(A, b);
    const int lane = lane_id();
    const int lev = PR == CclPred::Level ? wave >> 1 : 0;
    const bool right_edge = (wave & 1) == 0;
    if (PR == CclPred::Level && lev >= A.n_levels) return;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    int32_t *ids = A.ids + lev * nid;
    const int ntx = (A.w + CT - 1) / CT;
    auto tb = [&](int tx, int ty) -> const int32_t * { return border_table(A, lev, ty * ntx + tx); };
    int ra, rb, rbm1, rb64;
    if (right_edge) {   // a = this tile's right column, b = the right neighbour's left column, position = row
        if (t.x0 + CT >= A.w) return;
        ra = tb(t.tx, t.ty)[64 + lane];
        rb = tb(t.tx + 1, t.ty)[lane];
        rbm1 = t.y0 > 0 ? tb(t.tx + 1, t.ty - 1)[CT - 1] : -1;          // (x0 + 64, y0 - 1)
        rb64 = t.y0 + CT < A.h ? tb(t.tx + 1, t.ty + 1)[0] : -1;        // (x0 + 64, y0 + 64)
    } else {            // a = this tile's bottom row, b = the lower neighbour's top row, position = column
        if (t.y0 + CT >= A.h) return;
        ra = tb(t.tx, t.ty)[192 + lane];
        rb = tb(t.tx, t.ty + 1)[128 + lane];
        rbm1 = t.x0 > 0 ? tb(t.tx - 1, t.ty + 1)[128 + CT - 1] : -1;   // (x0 - 1, y0 + 64)
        rb64 = t.x0 + CT < A.w ? tb(t.tx + 1, t.ty + 1)[128] : -1;      // (x0 + 64, y0 + 64)
    }
    const uint64_t am = __ballot(ra >= 0), bm = __ballot(rb >= 0);
    const int rbl = __shfl(rb, lane > 0 ? lane - 1 : 0), rbr = __shfl(rb, lane < CT - 1 ? lane + 1 : CT - 1);
    edge_unions(ids, am, bm, rbm1 >= 0, rb64 >= 0, A.conn, lane, ra, lane > 0 ? rbl : rbm1, rb,
                lane < CT - 1 ? rbr : rb64);
}

// One workgroup per tile, one wave per (level, edge).
template <CclPred PR, CclOut OU>
__global__ __launch_bounds__(2 * CT * MAXLEV) void k_ccl_merge(const CclArgs *args, int n, int total) {
    const int wave = threadIdx.x / CT;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const CclArgs A = args[img_of(args, n, u)];
        ccl_merge_tile<PR>(A, u - A.unit0, wave);
    }
}

// ---------------------------------------------------------------------------
// flatten phase + outputs
// ---------------------------------------------------------------------------
// Sets, for every run start r, P[r] = -(global root id of its component) - 1.
// A component that does not reach the tile border is complete: its root is
// its global root.  The roots of the others are gathered into a list and
// looked up one per lane, so that their global finds overlap.
__device__ void resolve_roots(const CclArgs &A, const Tile &t, const WaveMem &M, const int32_t *ids, bool live) {
    const uint64_t *rows = M.rows;
    int *P = M.P;
    if (lane_id() == 0) *M.count = 0;
    mark_touch(t, rows, P);
    const int y = lane_id();
    const uint64_t m = live ? rows[y] : 0ull;
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const int s = __builtin_ctzll(st);
        const int li = y * CT + s;
        const int pv = P[slot(li)];
        if ((pv & LIDX) != li) continue;
        if (pv & TOUCH_BIT)
            M.list[atomicAdd(M.count, 1)] = li;
        else
            P[slot(li)] = -gid(A, t, s, y) - 1;
    }
    __syncthreads();
    const int nl = *M.count;
    for (int i = y; i < nl; i += CT) {
        const int li = M.list[i];
        P[slot(li)] = -gfind_ro(ids, gid(A, t, li & (CT - 1), li >> 6)) - 1;
    }
    __syncthreads();
    // the other runs copy their root's entry (roots are only read here)
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const int li = y * CT + __builtin_ctzll(st);
        const int r = P[slot(li)];
        if (r >= 0) P[slot(li)] = P[slot(r & LIDX)];
    }
    __syncthreads();
}

// global root of the run that starts at tile index li (after resolve_roots)
__device__ __forceinline__ int global_of_run(const int *P, int li) { return -P[slot(li)] - 1; }

__device__ __forceinline__ int global_of(const uint64_t *rows, const int *P, int x, int y) {
    return global_of_run(P, y * CT + run_start_of(rows[y], x));
}

// Stores 16 bytes (nvalid of them inside the image).
__device__ __forceinline__ void store16(uint8_t *p, const uint32_t w[4], int nvalid, bool wide) {
    if (wide && nvalid == 16) {
        *(uint4 *)p = make_uint4(w[0], w[1], w[2], w[3]);
        return;
    }
    for (int i = 0; i < nvalid; ++i) p[i] = (uint8_t)(w[i >> 2] >> ((i & 3) * 8));
}

// FillHoles and the multi-level bound need only the members whose component
// reaches the virtual frame node.  Such a component reaches the tile border,
// so its border pixels carry it: each run of a border row and each vertical
// run of a border column looks up its global root once (the local phase
// published every border pixel), the runs whose root is the frame node seed
// the set, and a flood inside the tile row masks completes it.  No forest is
// rebuilt.  The result rows go to the wave's LDS rows; wave l of the
// multi-level mode holds level l.
template <CclPred PR, CclOut OU>
__device__ __forceinline__ void ccl_flatten_fc_tile(const CclArgs &A, int b, int wave) {
    const Tile t = tile_of(A, b);
    const int lane = lane_id();
    const bool live = PR != CclPred::Level || wave < A.n_levels;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    uint64_t *rows = ccl_smem + wave * CT;
    build_rows<PR>(A, t, wave_level<PR>(A, wave), rows);
    const uint64_t m = rows[lane];
    const uint64_t top = rows[0], bot = rows[t.th - 1];
    const uint64_t above = lane > 0 ? rows[lane - 1] : 0ull;
    const int xr = t.tw - 1;
    // each border run's local root, from the border table, once per run
    int x[4] = {-1, -1, -1, -1};
    if (live) {
        const int32_t *bt = border_table(A, wave, b);
        if ((run_starts(top) >> lane) & 1ull) x[0] = bt[128 + lane];
        if (t.th > 1 && ((run_starts(bot) >> lane) & 1ull)) x[1] = bt[192 + lane];
        if ((m & 1ull) && !(above & 1ull)) x[2] = bt[lane];
        if (xr > 0 && ((m >> xr) & 1ull) && !((above >> xr) & 1ull)) x[3] = bt[64 + lane];
    }
    gfind4_ro(A.ids + (live ? wave : 0) * nid, x);
    const uint64_t s_top = __ballot(x[0] == 0), s_bot = __ballot(x[1] == 0);
    const uint64_t lcol = run_fill(__ballot(m & 1ull), __ballot(x[2] == 0));
    const uint64_t rcol = xr > 0 ? run_fill(__ballot((m >> xr) & 1ull), __ballot(x[3] == 0)) : 0ull;
    uint64_t f = ((lcol >> lane) & 1ull) | (((rcol >> lane) & 1ull) << xr);
    if (lane == 0) f |= s_top;
    if (lane == t.th - 1) f |= s_bot;
    f = flood_rows(m, f, A.conn);
    __syncthreads();
    rows[lane] = f;
    __syncthreads();

    const bool wide = OU == CclOut::LevelBound ? aligned16(A.bound, A.pitch_r) : aligned16(A.fill, A.pitch_f);
    const int nw = OU == CclOut::LevelBound ? blockDim.x / CT : 1;
    const int nlev = OU == CclOut::LevelBound ? min(nw, A.n_levels) : 0;
    for (int i = (int)threadIdx.x; i < CT * 4; i += nw * CT) {   // 16-pixel chunks
        const int y = i >> 2, c = i & 3;
        const int nvalid = y < t.th ? max(0, min(16, t.tw - 16 * c)) : 0;
        if (nvalid == 0) continue;
        const int64_t gy = t.y0 + y;
        const int gx = t.x0 + 16 * c;
        uint32_t w[4] = {0, 0, 0, 0};
        if constexpr (OU == CclOut::FillHoles) {
            // F = input | not frame-connected: members of the background
            // components that reach the frame are the only zeros
            const uint32_t fc = ~(uint32_t)(rows[y] >> (16 * c));
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = nibble_bytes(fc >> (4 * q));
            store16(A.fill + gy * A.pitch_f + gx, w, nvalid, wide);
        } else {
            if (gy == 0 || gy == A.h - 1) {
                // a frame row: the frame marker J = Hq, which is also the
                // bound there (a frame pixel joins every level set it is in)
                const uint4 q = load16(A.a + gy * A.pitch_a + gx, nvalid, aligned16(A.a, A.pitch_a));
                w[0] = q.x;
                w[1] = q.y;
                w[2] = q.z;
                w[3] = q.w;
            } else {
                // the highest level whose frame-connected set holds the
                // pixel: the level sets are nested and the levels come in
                // non-decreasing order, so each level overwrites the bytes
                // of its set
                for (int l = 0; l < nlev; ++l) {
                    const uint32_t f = (uint32_t)(ccl_smem[l * CT + y] >> (16 * c));
                    const uint32_t L = (uint32_t)A.levels[l] * 0x01010101u;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t b = nibble_bytes(f >> (4 * q)) * 0xffu;
                        w[q] = (b & L) | (~b & w[q]);
                    }
                }
                // frame columns: J = Hq
                auto put = [&](int k) {
                    const uint32_t v = A.a[gy * A.pitch_a + gx + k];
                    const int sh = (k & 3) * 8;
                    w[k >> 2] = (w[k >> 2] & ~(0xffu << sh)) | (v << sh);
                };
                if (gx == 0) put(0);
                const int kr = A.w - 1 - gx;
                if (kr >= 0 && kr < nvalid) put(kr);
            }
            store16(A.bound + gy * A.pitch_r + gx, w, nvalid, wide);
        }
    }
}

__device__ void tile_stats(const CclArgs &A, const Tile &t, const uint64_t *rows, const int *P);
__device__ void write_labels(const CclArgs &A, const Tile &t, const uint64_t *rows, const int *P);

// BWLabel output: labels, the cleared output mask, and the per-component
// statistics.  A tile's runs are first summed per component in
// an LDS table (a few entries per tile), so each component costs one set of
// global atomics per tile instead of one per run; components are registered
// with one counter update per wave.
__device__ __forceinline__ void ccl_flatten_labels_tile(const CclArgs &A, int b) {
    const Tile t = tile_of(A, b);
    const WaveMem M = wave_mem(0);
    uint64_t *rows = M.rows;
    int *P = M.P;
    build_rows<CclPred::NonZero>(A, t, 0, rows);
    run_forest(rows, P, A.conn);
    resolve_roots(A, t, M, A.ids, true);
    // statistics first: the list registration waits for its counter, and
    // that wait (one count of vector memory operations) also covers every
    // store issued before it
    if (A.st_area || A.obj_list) tile_stats(A, t, rows, P);
    write_labels(A, t, rows, P);
}

// Per-component area, bounding box and registration of the tile's roots.
__device__ void tile_stats(const CclArgs &A, const Tile &t, const uint64_t *rows, const int *P) {
    const int lane = lane_id();
    int *key = wave_mem(0).list;   // the root list is no longer needed
    int *area = key + NHASH, *x0 = area + NHASH, *x1 = x0 + NHASH, *y0 = x1 + NHASH, *y1 = y0 + NHASH;
    for (int i = lane; i < NHASH; i += CT) {
        key[i] = -1;
        area[i] = 0;
        x0[i] = 0x7fffffff;
        x1[i] = -1;
        y0[i] = 0x7fffffff;
        y1[i] = -1;
    }
    __syncthreads();
    // per run (lane = row)
    const int y = lane;
    const uint64_t m = rows[y];
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const int s = __builtin_ctzll(st);
        const int len = run_len(m, s);
        const int g = global_of_run(P, y * CT + s);
        const bool is_root = g == gid(A, t, s, y);
        int k = (int)(((uint32_t)g * 2654435761u) >> 25) & (NHASH - 1);
        bool ok = false;
        for (int probe = 0; probe < NHASH; ++probe) {
            const int old = atomicCAS(key + k, -1, g);
            if (old == -1 || old == g) {
                ok = true;
                break;
            }
            k = (k + 1) & (NHASH - 1);
        }
        if (ok) {
            atomicAdd(area + k, len);
            atomicMin(x0 + k, t.x0 + s);
            atomicMax(x1 + k, t.x0 + s + len - 1);
            atomicMin(y0 + k, t.y0 + y);
            atomicMax(y1 + k, t.y0 + y);
            if (is_root) atomicOr(area + k, ROOT_FLAG);
        } else {   // table full: this run goes to global memory directly
            if (A.st_area) {
                atomicAdd(A.st_area + g, len);
                atomicMin(A.st_x0 + g, t.x0 + s);
                atomicMax(A.st_x1 + g, t.x0 + s + len - 1);
                atomicMin(A.st_y0 + g, t.y0 + y);
                atomicMax(A.st_y1 + g, t.y0 + y);
            }
            if (A.obj_list && is_root) A.obj_list[atomicAdd(A.n_obj, 1)] = (A.img << 25) | g;
        }
    }
    __syncthreads();
    for (int i = lane; i < NHASH; i += CT) {
        const int g = key[i];
        bool r = false;
        if (g >= 0) {
            const int ar = area[i];
            if (A.st_area) {
                atomicAdd(A.st_area + g, ar & ~ROOT_FLAG);
                atomicMin(A.st_x0 + g, x0[i]);
                atomicMax(A.st_x1 + g, x1[i]);
                atomicMin(A.st_y0 + g, y0[i]);
                atomicMax(A.st_y1 + g, y1[i]);
            }
            r = A.obj_list && (ar & ROOT_FLAG);
        }
        const uint64_t bm = __ballot(r);
        if (bm) {
            int base = 0;
            if (lane == 0) base = atomicAdd(A.n_obj, __popcll(bm));
            base = __shfl(base, 0);
            if (r) A.obj_list[base + __popcll(bm & ((1ull << lane) - 1))] = (A.img << 25) | g;
        }
    }
}

// Labels of the tile, 16 bytes per lane and row: lane = group of 4 columns
// (lane % 16) and row phase (lane / 16), so that one store covers 4 rows.
// The mask is cleared over the whole tile with 16-byte stores; the
// per-object stage writes every member pixel afterwards.
__device__ void write_labels(const CclArgs &A, const Tile &t, const uint64_t *rows, const int *P) {
    const int lane = lane_id();
    const int x4 = 4 * (lane & 15);
    const int nv = max(0, min(4, t.tw - x4));
    const bool wide = aligned16(A.labels, A.pitch_l * (int64_t)sizeof(int32_t));
    for (int y = lane >> 4; y < t.th; y += 4) {
        const uint64_t m = rows[y];
        const uint32_t g4 = (uint32_t)(m >> x4) & 15u;
        // run start of each of the 4 pixels (any column for a non-member):
        // a member continues its left neighbour's run or starts one
        int rs[4];
        rs[0] = (g4 & 1u) ? run_start_of(m, x4) : x4;
#pragma unroll
        for (int j = 1; j < 4; ++j) rs[j] = ((g4 >> (j - 1)) & 1u) ? rs[j - 1] : x4 + j;
        int v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = global_of_run(P, y * CT + rs[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = ((g4 >> j) & 1u) ? v[j] : 0;
        int32_t *dst = A.labels + (t.y0 + y) * A.pitch_l + t.x0 + x4;
        if (wide && nv == 4) {
            *(int4 *)dst = make_int4(v[0], v[1], v[2], v[3]);
        } else {
            for (int j = 0; j < nv; ++j) dst[j] = v[j];
        }
    }
    if (A.zero_mask) {
        const int c = lane & 3;
        const int nvm = max(0, min(16, t.tw - 16 * c));
        const bool wm = aligned16(A.zero_mask, A.pitch_m);
        const uint32_t z[4] = {0, 0, 0, 0};
        for (int y = lane >> 2; y < t.th; y += 16) store16(A.zero_mask + (t.y0 + y) * A.pitch_m + t.x0 + 16 * c, z, nvm, wm);
    }
}

template <CclPred PR, CclOut OU>
__global__ __launch_bounds__(CT * MAXLEV) void k_ccl_flatten(const CclArgs *args, int n, int total) {
    const int wave = threadIdx.x / CT;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const CclArgs A = args[img_of(args, n, u)];
        if constexpr (OU == CclOut::Labels)
            ccl_flatten_labels_tile(A, u - A.unit0);
        else
            ccl_flatten_fc_tile<PR, OU>(A, u - A.unit0, wave);
        __syncthreads();
    }
}

int ccl_tiles(int w, int h) { return ((w + CT - 1) / CT) * ((h + CT - 1) / CT); }

template <CclPred PR, CclOut OU>
static int launch_ccl_t(const CclArgs *args_dev, int n, int total, int n_cu, hipStream_t s, int nw) {
    const size_t lds_flat = OU == CclOut::Labels ? (size_t)LABELS_LDS : (size_t)nw * CT * 8;
    const int cap = n_cu * 128;
    hipLaunchKernelGGL((k_ccl_local<PR, OU>), dim3(std::min(total * nw, cap)), dim3(CT), LOCAL_LDS, s, args_dev, n,
                       total, nw);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_ccl_merge<PR, OU>), dim3(std::min(total, cap)), dim3(2 * CT * nw), 0, s, args_dev, n, total);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_ccl_flatten<PR, OU>), dim3(std::min(total, cap)), dim3(CT * nw), lds_flat, s, args_dev, n,
                       total);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_ccl(const CclArgs *args_dev, int n, int total, int n_cu, hipStream_t s, CclPred pred, CclOut out,
               int n_levels) {
    if (total <= 0) return RT_OK;
    if (pred == CclPred::Level && out == CclOut::LevelBound) {
        if (n_levels < 1 || n_levels > MAXLEV) {
            set_error("ccl: %d threshold levels (1..%d)", n_levels, MAXLEV);
            return RT_EINVAL;
        }
        return launch_ccl_t<CclPred::Level, CclOut::LevelBound>(args_dev, n, total, n_cu, s, n_levels);
    }
    if (pred == CclPred::TophatBg && out == CclOut::FillHoles)
        return launch_ccl_t<CclPred::TophatBg, CclOut::FillHoles>(args_dev, n, total, n_cu, s, 1);
    if (pred == CclPred::Zero && out == CclOut::FillHoles)
        return launch_ccl_t<CclPred::Zero, CclOut::FillHoles>(args_dev, n, total, n_cu, s, 1);
    if (pred == CclPred::NonZero && out == CclOut::Labels)
        return launch_ccl_t<CclPred::NonZero, CclOut::Labels>(args_dev, n, total, n_cu, s, 1);
    set_error("ccl: unsupported predicate / output pair");
    return RT_EUNSUPPORTED;
}

}  // namespace rtseg
