// Connected-component labelling by union-find (BWLabel, Sec. 5.1: a forest
// in which every pixel starts as its own tree, adjacent trees are merged, and
// labels are read off by flattening the trees).
//
// One wavefront per 64 x 64 tile.  A row of the tile is one 64-bit ballot
// mask, so the forest is built over horizontal runs instead of pixels: the
// pixels of a run share its first pixel as parent by construction (bit
// arithmetic, no atomics), and only runs of adjacent rows that touch are
// united (LDS atomicMin, the root is always the smallest index, so labels are
// canonical by construction).  Three launches:
//   local  : build the tile forest; publish only its roots and its edge
//            pixels to the global id array (id 0 = virtual node, pixel p has
//            id p + 1);
//   merge  : one wave per tile unites, across its right and bottom edges,
//            each pair of touching edge runs once (global atomicMin);
//   flatten: rebuild the tile forest (it costs 1 byte/pixel of input instead
//            of 4 bytes/pixel of stored local roots), find each local root's
//            global root once, and write the per-pixel result.
// Modes: BWLabel (labels, per-component area and bounding box, component
// list), FillHoles (background components joined to a virtual frame node),
// and the multi-level frame-connectivity lower bound that starts the
// grayscale reconstruction.
#include "rt_internal.h"

namespace rtseg {

constexpr int CT = 64;                 // tile edge = wavefront size
constexpr int MAXLEV = 8;
constexpr int FRAME_BIT = 1 << 30;     // tags a local root whose component touches the image frame
constexpr int TOUCH_BIT = 1 << 29;     // tags a local root whose component touches the tile border
constexpr int LIDX = 0xfff;

__device__ __forceinline__ int ld_agent(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Finds with path halving: a node is re-pointed to its grandparent with
// atomicMin, so parent pointers only ever move to a smaller ancestor and a
// concurrent link can never be undone.
__device__ __forceinline__ int lfind(int *P, int x) {
    int p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        const int gp = __hip_atomic_load(P + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (gp != p) atomicMin(P + x, gp);
        x = p;
        p = gp;
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
        int old = atomicMin(P + a, b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ int gfind(int32_t *ids, int x) {
    int p = ld_agent(ids + x);
    while (p != x) {
        const int gp = ld_agent(ids + p);
        if (gp != p) atomicMin(ids + x, gp);
        x = p;
        p = gp;
    }
    return x;
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
__device__ __forceinline__ uint64_t bits_upto(int e) { return e >= 63 ? ~0ull : (2ull << e) - 1; }

// ---- predicate --------------------------------------------------------------
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

// Column `lane` of the tile, held by that lane: predicate bits (non-Level
// modes) or the packed uint8 values (Level mode), 4 per word.
struct Col {
    uint32_t v[16];
};

__device__ void load_col(const CclArgs &A, const Tile &t, Col &c) {
    const int lane = threadIdx.x;
    const int x = t.x0 + lane;
#pragma unroll
    for (int k = 0; k < 16; ++k) c.v[k] = 0;
    if (lane >= t.tw) return;
#pragma unroll
    for (int y = 0; y < CT; ++y) {
        if (y < t.th) {
            uint32_t v;
            if (A.pred == CclPred::Level)
                v = A.a[(int64_t)(t.y0 + y) * A.pitch_a + x];
            else
                v = eval_pred(A, x, t.y0 + y, 0) ? 1u : 0u;
            c.v[y >> 2] |= v << ((y & 3) * 8);
        }
    }
}

__device__ __forceinline__ bool col_bit(const CclArgs &A, const Col &c, int y, int level) {
    uint32_t v = (c.v[y >> 2] >> ((y & 3) * 8)) & 255u;
    return A.pred == CclPred::Level ? (int)v >= level : v != 0;
}

// rows[y] = ballot over lanes (= columns) of the member bit at row y
__device__ void make_rows(const CclArgs &A, const Tile &t, const Col &c, int level, uint64_t *rows) {
    const int lane = threadIdx.x;
    uint64_t mine = 0;
#pragma unroll
    for (int y = 0; y < CT; ++y) {
        bool b = y < t.th && lane < t.tw && col_bit(A, c, y, level);
        uint64_t m = __ballot(b);
        if (lane == y) mine = m;
    }
    rows[lane] = mine;
    __syncthreads();
}

// Tile forest over runs: after the call, P[y*64+s] = local root (index of a
// run start) for every run start s of row y.  Lane = row.
__device__ void run_forest(const uint64_t *rows, int *P, int conn) {
    const int y = threadIdx.x;
    const uint64_t m = rows[y];
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        int s = __builtin_ctzll(st);
        P[y * CT + s] = y * CT + s;
    }
    __syncthreads();
    if (y > 0) {
        const uint64_t pm = rows[y - 1];
        if (m && pm) {
            for (uint64_t st = run_starts(m); st; st &= st - 1) {
                int s = __builtin_ctzll(st);
                int e = s + run_len(m, s) - 1;
                int lo = conn == 8 ? max(s - 1, 0) : s;
                int hi = conn == 8 ? min(e + 1, 63) : e;
                uint64_t ov = pm & bits_upto(hi) & ~((1ull << lo) - 1);
                while (ov) {
                    int b = __builtin_ctzll(ov);
                    int s2 = run_start_of(pm, b);
                    int e2 = s2 + run_len(pm, s2) - 1;
                    lunite(P, y * CT + s, (y - 1) * CT + s2);
                    ov &= ~bits_upto(e2);
                }
            }
        }
    }
    __syncthreads();
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        int s = __builtin_ctzll(st);
        P[y * CT + s] = lfind(P, y * CT + s);
    }
    __syncthreads();
}

__device__ __forceinline__ int root_of(const uint64_t *rows, const int *P, int x, int y) {
    return P[y * CT + run_start_of(rows[y], x)] & LIDX;
}

// Tags the roots of components that reach the tile border.  Only those can
// be joined to other tiles; a component that touches the image frame touches
// the tile border too.  Lane = row.
__device__ void mark_touch(const Tile &t, const uint64_t *rows, int *P) {
    const int y = threadIdx.x;
    const uint64_t m = rows[y];
    if (y < t.th && m) {
        if (y == 0 || y == t.th - 1) {
            for (uint64_t st = run_starts(m); st; st &= st - 1)
                atomicOr(P + (P[y * CT + __builtin_ctzll(st)] & LIDX), TOUCH_BIT);
        } else {
            if (m & 1ull) atomicOr(P + root_of(rows, P, 0, y), TOUCH_BIT);
            if ((m >> (t.tw - 1)) & 1ull) atomicOr(P + root_of(rows, P, t.tw - 1, y), TOUCH_BIT);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// local phase
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ccl_local_tile(const CclArgs &A, int b, uint64_t *rows, int *P);

__global__ __launch_bounds__(CT) void k_ccl_local(const CclArgs *args, int n, int total) {
    __shared__ uint64_t rows[CT];
    __shared__ int P[CT * CT];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const CclArgs A = args[img_of(args, n, u)];
        ccl_local_tile(A, u - A.unit0, rows, P);
    }
}

__device__ __forceinline__ void ccl_local_tile(const CclArgs &A, int b, uint64_t *rows, int *P) {
    const Tile t = tile_of(A, b);
    const int lane = threadIdx.x;
    if (b == 0 && lane == 0) {  // the virtual node of every level is its own root
        const int nl = A.pred == CclPred::Level ? A.n_levels : 1;
        for (int l = 0; l < nl; ++l) A.ids[(int64_t)l * ((int64_t)A.w * A.h + 1)] = 0;
    }
    Col c;
    load_col(A, t, c);
    const int nlev = A.pred == CclPred::Level ? A.n_levels : 1;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    const bool tile_on_frame = t.x0 == 0 || t.y0 == 0 || t.x0 + t.tw == A.w || t.y0 + t.th == A.h;
    for (int lev = 0; lev < nlev; ++lev) {
        const int level = A.pred == CclPred::Level ? A.levels[lev] : 0;
        int32_t *ids = A.ids + lev * nid;
        make_rows(A, t, c, level, rows);
        run_forest(rows, P, A.conn);
        mark_touch(t, rows, P);
        const int y = lane;
        const uint64_t m = rows[y];
        if (A.frame_virtual && tile_on_frame) {
            if (y < t.th && m) {
                if (t.y0 + y == 0 || t.y0 + y == A.h - 1) {
                    for (uint64_t st = run_starts(m); st; st &= st - 1)
                        atomicOr(P + (P[y * CT + __builtin_ctzll(st)] & LIDX), FRAME_BIT);
                } else {
                    if (t.x0 == 0 && (m & 1ull)) atomicOr(P + root_of(rows, P, 0, y), FRAME_BIT);
                    if (t.x0 + t.tw == A.w && ((m >> (t.tw - 1)) & 1ull))
                        atomicOr(P + root_of(rows, P, t.tw - 1, y), FRAME_BIT);
                }
            }
            __syncthreads();
        }
        // roots (lane = row)
        for (uint64_t st = run_starts(m); st; st &= st - 1) {
            int s = __builtin_ctzll(st);
            int li = y * CT + s;
            int pv = P[li];
            if ((pv & LIDX) != li) continue;
            int id = gid(A, t, s, y);
            if (pv & TOUCH_BIT) ids[id] = (pv & FRAME_BIT) ? 0 : id;
            if (A.st_area) {
                A.st_area[id] = 0;
                A.st_x0[id] = 0x7fffffff;
                A.st_y0[id] = 0x7fffffff;
                A.st_x1[id] = -1;
                A.st_y1[id] = -1;
            }
        }
        // edge pixels that are not roots: left / right columns (lane = row)
        if (m & 1ull) {
            int r = root_of(rows, P, 0, y);
            if (r != y * CT) ids[gid(A, t, 0, y)] = gid(A, t, r & 63, r >> 6);
        }
        if (t.tw > 1 && ((m >> (t.tw - 1)) & 1ull)) {
            int r = root_of(rows, P, t.tw - 1, y);
            int li = y * CT + t.tw - 1;
            if (r != li) ids[gid(A, t, t.tw - 1, y)] = gid(A, t, r & 63, r >> 6);
        }
        // top / bottom rows (lane = column)
        {
            const int x = lane;
            if ((rows[0] >> x) & 1ull) {
                int r = root_of(rows, P, x, 0);
                if (r != x) ids[gid(A, t, x, 0)] = gid(A, t, r & 63, r >> 6);
            }
            const int yb = t.th - 1;
            if (yb > 0 && ((rows[yb] >> x) & 1ull)) {
                int r = root_of(rows, P, x, yb);
                if (r != yb * CT + x) ids[gid(A, t, x, yb)] = gid(A, t, r & 63, r >> 6);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// merge phase: one wave per tile, its right and bottom edges
// ---------------------------------------------------------------------------
// unites the pairs (a(i), b(i+d)), d in {-1,0,1} (8-conn) or {0} (4-conn),
// along an edge; a/b bit i = member at position i (b has two extra members
// at i = -1 and i = 64, passed as bm1 / b64; they lie in the diagonal
// neighbour tiles).  About one union per pair of touching runs: a pair is
// skipped when a pair with a lower position, together with an adjacency
// inside one tile (always joined by that tile's forest), implies it.
__device__ void edge_unions(int32_t *ids, uint64_t am, uint64_t bm, bool bm1, bool b64, int conn, int i,
                            int ida, int idb_base, int idb_stride) {
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
        gunite(ids, ida, idb_base + i * idb_stride);
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
        gunite(ids, ida, idb_base + j * idb_stride);
    }
}

__device__ __forceinline__ void ccl_merge_tile(const CclArgs &A, int b);

__global__ __launch_bounds__(CT) void k_ccl_merge(const CclArgs *args, int n, int total) {
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const CclArgs A = args[img_of(args, n, u)];
        ccl_merge_tile(A, u - A.unit0);
    }
}

__device__ __forceinline__ void ccl_merge_tile(const CclArgs &A, int b) {
    const Tile t = tile_of(A, b);
    const int lane = threadIdx.x;
    const int nlev = A.pred == CclPred::Level ? A.n_levels : 1;
    const int64_t nid = (int64_t)A.w * A.h + 1;
    const bool right = t.x0 + CT < A.w;
    const bool bottom = t.y0 + CT < A.h;
    if (!right && !bottom) return;
    for (int lev = 0; lev < nlev; ++lev) {
        const int level = A.pred == CclPred::Level ? A.levels[lev] : 0;
        int32_t *ids = A.ids + lev * nid;
        if (right) {   // a = column x0+63, b = column x0+64, position = row
            const int xa = t.x0 + CT - 1, xb = t.x0 + CT;
            bool a = lane < t.th && eval_pred(A, xa, t.y0 + lane, level);
            bool b = lane < t.th && eval_pred(A, xb, t.y0 + lane, level);
            uint64_t am = __ballot(a), bm = __ballot(b);
            bool bm1 = t.y0 > 0 && eval_pred(A, xb, t.y0 - 1, level);
            bool b64 = t.y0 + CT < A.h && eval_pred(A, xb, t.y0 + CT, level);
            if (lane < t.th)
                edge_unions(ids, am, bm, bm1, b64, A.conn, lane, (t.y0 + lane) * A.w + xa + 1,
                            t.y0 * A.w + xb + 1, A.w);
        }
        if (bottom) {  // a = row y0+63, b = row y0+64, position = column
            const int ya = t.y0 + CT - 1, yb = t.y0 + CT;
            bool a = lane < t.tw && eval_pred(A, t.x0 + lane, ya, level);
            bool b = lane < t.tw && eval_pred(A, t.x0 + lane, yb, level);
            uint64_t am = __ballot(a), bm = __ballot(b);
            bool bm1 = t.x0 > 0 && eval_pred(A, t.x0 - 1, yb, level);
            bool b64 = t.x0 + CT < A.w && eval_pred(A, t.x0 + CT, yb, level);
            if (lane < t.tw)
                edge_unions(ids, am, bm, bm1, b64, A.conn, lane, ya * A.w + t.x0 + lane + 1, yb * A.w + t.x0 + 1, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// flatten phase + outputs
// ---------------------------------------------------------------------------
// Replaces, for every local root r, P[r] by -(global root id) - 1.  A
// component that does not reach the tile border is complete: its root is
// its global root.  The others look theirs up.
__device__ void resolve_roots(const CclArgs &A, const Tile &t, const uint64_t *rows, int *P, int32_t *ids) {
    mark_touch(t, rows, P);
    const int y = threadIdx.x;
    const uint64_t m = rows[y];
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const int s = __builtin_ctzll(st);
        const int li = y * CT + s;
        const int pv = P[li];
        if ((pv & LIDX) != li) continue;
        const int id = gid(A, t, s, y);
        P[li] = -((pv & TOUCH_BIT) ? gfind_ro(ids, id) : id) - 1;
    }
    __syncthreads();
}

__device__ __forceinline__ int global_of(const uint64_t *rows, const int *P, int x, int y) {
    int r = P[y * CT + run_start_of(rows[y], x)];
    if (r < 0) return -r - 1;
    return -P[r] - 1;
}

__device__ __forceinline__ void ccl_flatten_tile(const CclArgs &A, int b, uint64_t *rows, int *P);

__global__ __launch_bounds__(CT) void k_ccl_flatten(const CclArgs *args, int n, int total) {
    __shared__ uint64_t rows[CT];
    __shared__ int P[CT * CT];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const CclArgs A = args[img_of(args, n, u)];
        ccl_flatten_tile(A, u - A.unit0, rows, P);
        __syncthreads();
    }
}

__device__ __forceinline__ void ccl_flatten_tile(const CclArgs &A, int b, uint64_t *rows, int *P) {
    const Tile t = tile_of(A, b);
    const int lane = threadIdx.x;
    Col c;
    load_col(A, t, c);
    const int64_t nid = (int64_t)A.w * A.h + 1;
    const int x = lane;

    if (A.out == CclOut::LevelBound) {
        uint32_t best[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) best[k] = 0;
        for (int lev = 0; lev < A.n_levels; ++lev) {
            const int level = A.levels[lev];
            make_rows(A, t, c, level, rows);
            run_forest(rows, P, A.conn);
            resolve_roots(A, t, rows, P, A.ids + lev * nid);
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                if (y >= t.th || !((rows[y] >> x) & 1ull)) continue;
                if (global_of(rows, P, x, y) != 0) continue;
                const uint32_t cur = (best[y >> 2] >> ((y & 3) * 8)) & 255u;
                if ((uint32_t)level > cur)
                    best[y >> 2] = (best[y >> 2] & ~(255u << ((y & 3) * 8))) | ((uint32_t)level << ((y & 3) * 8));
            }
            __syncthreads();
        }
        if (x < t.tw) {
            const int gx = t.x0 + x;
#pragma unroll
            for (int y = 0; y < CT; ++y) {
                if (y >= t.th) continue;
                const int gy = t.y0 + y;
                int v = (best[y >> 2] >> ((y & 3) * 8)) & 255;
                if (gx == 0 || gy == 0 || gx == A.w - 1 || gy == A.h - 1) {
                    int j = (c.v[y >> 2] >> ((y & 3) * 8)) & 255;   // frame marker J = Hq
                    v = v > j ? v : j;
                }
                A.bound[(int64_t)gy * A.pitch_r + gx] = (uint8_t)v;
            }
        }
        return;
    }

    make_rows(A, t, c, 0, rows);
    run_forest(rows, P, A.conn);
    resolve_roots(A, t, rows, P, A.ids);
    if (x < t.tw) {
        const int gx = t.x0 + x;
        for (int y = 0; y < t.th; ++y) {
            const int64_t gy = t.y0 + y;
            const bool mem = (rows[y] >> x) & 1ull;
            if (A.out == CclOut::Labels) {
                A.labels[gy * A.pitch_l + gx] = mem ? global_of(rows, P, x, y) : 0;
                if (!mem && A.bg_zero_mask) A.bg_zero_mask[gy * A.pitch_m + gx] = 0;
            } else {  // FillHoles: members are background pixels of the input
                A.fill[gy * A.pitch_f + gx] = mem ? (global_of(rows, P, x, y) != 0 ? 1 : 0) : 1;
            }
        }
    }
    if (A.out != CclOut::Labels || (!A.st_area && !A.obj_list)) return;
    // per-run statistics and component registration (lane = row)
    const int y = lane;
    const uint64_t m = rows[y];
    for (uint64_t st = run_starts(m); st; st &= st - 1) {
        const int s = __builtin_ctzll(st);
        const int len = run_len(m, s);
        const int g = global_of(rows, P, s, y);
        if (A.st_area) {
            atomicAdd(A.st_area + g, len);
            atomicMin(A.st_x0 + g, t.x0 + s);
            atomicMax(A.st_x1 + g, t.x0 + s + len - 1);
            atomicMin(A.st_y0 + g, t.y0 + y);
            atomicMax(A.st_y1 + g, t.y0 + y);
        }
        if (A.obj_list && P[y * CT + s] < 0 && g == gid(A, t, s, y))
            A.obj_list[atomicAdd(A.n_obj, 1)] = (A.img << 25) | g;
    }
}

int ccl_tiles(int w, int h) { return ((w + CT - 1) / CT) * ((h + CT - 1) / CT); }

int launch_ccl(const CclArgs *args_dev, int n, int total, int n_cu, hipStream_t s) {
    if (total <= 0) return RT_OK;
    const int grid = std::min(total, n_cu * 16);
    hipLaunchKernelGGL(k_ccl_local, dim3(grid), dim3(CT), 0, s, args_dev, n, total);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ccl_merge, dim3(grid), dim3(CT), 0, s, args_dev, n, total);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ccl_flatten, dim3(grid), dim3(CT), 0, s, args_dev, n, total);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rtseg
