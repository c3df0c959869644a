// Pre-Watershed + Watershed, one wavefront per connected component.
//
// The paper restructures feature computation into one bounding box per
// nucleus, one GPU block per box (Sec. 5.1); the same decomposition serves
// the watershed stage here.  Everything after the first area filter
// (distance transform, h-maxima seeds, flood, cut, relabelling, final area
// filter) depends only on the component itself:
//   * the nearest background pixel of a component pixel lies in the
//     component's bounding box grown by one pixel (the open disc of radius d
//     around p holds no background pixel, so it is a connected foreground set
//     inside the component, and the background pixel that ends the disc is
//     8-adjacent to the component), so the distance transform of the crop with
//     "not in the component" as background is exact;
//   * the reconstructions run on the graph of the component's own pixels, and
//     different components are never 8-adjacent.
// A component with at most one seed is labelled whole (every pixel can only
// take that seed's label), so the flood runs only for touching nuclei.
//
// Crop planes (row stride odd, so a column walk does not hit one LDS bank):
//   fl  flags: in component / seed / kept
//   dq  Dq, later the level-sorted list of unlabelled pixels, later areas
//   A   g (h-maxima), then lambda, then CCL roots of the kept pixels
//   B   recon of g-1 under g, then labels; during one flood level a pixel of
//       that level holds -(key) - 2 with key = (BFS distance << SH) | label
// Size classes: crops of at most 32 x 32 and 64 x 64 pixels live in LDS (one
// wave per component, many components per CU) and run their reconstructions
// with the crop in registers; larger crops use a global scratch slice with
// 64-bit keys.  All three launches read their work lists from device
// counters, so no host round trip is needed.
#include "crop_addr.h"
#include "rt_internal.h"

#include <climits>

namespace rtseg {

constexpr int WAVE = 64;
constexpr int RS_ = 32;                 // small class: crop <= 32 x 32
constexpr int RM_ = 64;                 // medium class: crop <= 64 x 64
constexpr int CAP_S = (RS_ + 1) * RS_;  // plane size with the odd row stride
constexpr int CAP_M = (RM_ + 1) * RM_;
constexpr int CAP_L = 97 * 96;           // large class: crops of at most 9312 px (about 96 x 96) in LDS
constexpr int HBINS = 256;
constexpr int NEGV = INT_MIN;
constexpr int GINF = 1 << 28;

enum : uint8_t { F_IN = 1, F_RM = 2, F_M = 4 };

template <typename L>
struct KeyPack;
template <>
struct KeyPack<int32_t> {  // crop plane < 65536 pixels: distance and label in 16 bits each
    static constexpr int SH = 16;
};
template <>
struct KeyPack<int64_t> {
    static constexpr int SH = 32;
};

template <typename L>
struct Crop {
    uint8_t *fl;
    int32_t *dq;
    int32_t *A;
    L *B;
    int st, cw, ch, cx0, cy0, n;
};

__device__ __forceinline__ int isqrt_exact(int64_t v) {
    if (v <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (int)r;
}

__device__ __forceinline__ bool wave_or(bool b) { return __syncthreads_or(b) != 0; }

// Within one wave: the hardware performs a wavefront's LDS operations in
// order, so it suffices that every earlier LDS access has completed and that
// the compiler moves no memory access across this point (a lane reads what
// other lanes of the wave wrote, which per-thread alias analysis cannot see).
__device__ __forceinline__ void wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// Barrier between the passes over an LDS crop plane (32-bit labels).  A
// one-wave workgroup needs no s_barrier, and no wait for its global stores
// (which a workgroup barrier implies): the wave's own LDS operations are
// performed in order.  Planes in global scratch (64-bit labels) keep the
// workgroup barrier, whose wait orders the wave's global stores and loads.
template <typename L>
__device__ __forceinline__ void crop_sync() {
    if (sizeof(L) == 4 && blockDim.x == WAVE)
        wave_sync();
    else
        __syncthreads();
}
template <typename L>
__device__ __forceinline__ bool crop_any(bool b) {
    if (sizeof(L) == 4 && blockDim.x == WAVE) {
        wave_sync();
        return __any(b) != 0;
    }
    return __syncthreads_or(b) != 0;
}

__device__ int wave_max(int v, int *red) {
    if (threadIdx.x == 0) *red = NEGV;
    __syncthreads();
    if (v != NEGV) atomicMax(red, v);
    __syncthreads();
    int r = *red;
    __syncthreads();
    return r;
}
__device__ int wave_min(int v, int *red) {
    if (threadIdx.x == 0) *red = INT_MAX;
    __syncthreads();
    if (v != INT_MAX) atomicMin(red, v);
    __syncthreads();
    int r = *red;
    __syncthreads();
    return r;
}

// ---- union-find on a crop plane (roots are the smallest index) -----------
// path halving with atomicMin: parents only move to smaller ancestors
template <typename T>
__device__ __forceinline__ T pfind(T *P, T x) {
    T p = __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (p != x) {
        const T gp = __hip_atomic_load(P + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (gp != p) __hip_atomic_fetch_min(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = p;
        p = gp;
    }
    return x;
}
template <typename T>
__device__ __forceinline__ void punite(T *P, T a, T b) {
    for (;;) {
        a = pfind(P, a);
        b = pfind(P, b);
        if (a == b) return;
        if (a < b) {
            T t = a;
            a = b;
            b = t;
        }
        T old = __hip_atomic_fetch_min(P + a, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
}

// P[i] = smallest index of the 8-connected component of flagged pixels, -1 elsewhere
template <typename L, typename T>
__device__ void crop_ccl(const Crop<L> &m, uint8_t bit, T *P) {
    for (int i = threadIdx.x; i < m.n; i += blockDim.x) P[i] = (m.fl[i] & bit) ? (T)i : (T)-1;
    __syncthreads();
    for (int i = threadIdx.x; i < m.n; i += blockDim.x) {
        if (!(m.fl[i] & bit)) continue;
        int c = i % m.st, r = i / m.st;
        if (c > 0 && (m.fl[i - 1] & bit)) punite<T>(P, i, i - 1);
        if (r > 0) {
            if (m.fl[i - m.st] & bit) punite<T>(P, i, i - m.st);
            if (c > 0 && (m.fl[i - m.st - 1] & bit)) punite<T>(P, i, i - m.st - 1);
            if (c < m.cw - 1 && (m.fl[i - m.st + 1] & bit)) punite<T>(P, i, i - m.st + 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m.n; i += blockDim.x)
        if (m.fl[i] & bit) P[i] = pfind<T>(P, (T)i);
    __syncthreads();
}

// ---- reconstruction by directional scans -----------------------------------
// V <- recon of V under M on the component's 8-connected graph.  Pixels
// outside the component hold NEGV in V and never change.  One sweep is four
// scans (down, up with lane = column; right, left with lane = row); within a
// scan each row/column reads its predecessor already updated.
template <typename L, typename V>
__device__ __forceinline__ bool relax1(const Crop<L> &m, V *val, const int32_t *M, int r, int c) {
    const int i = r * m.st + c;
    if (!(m.fl[i] & F_IN)) return false;
    // neighbours outside the crop are clamped onto in-crop pixels: repeating
    // a value (or the pixel itself) cannot change a maximum
    const int up = r > 0 ? -m.st : 0, dn = r < m.ch - 1 ? m.st : 0;
    const int lf = c > 0 ? -1 : 0, rt = c < m.cw - 1 ? 1 : 0;
    const V v0 = val[i + up + lf], v1 = val[i + up], v2 = val[i + up + rt];
    const V v3 = val[i + lf], v4 = val[i + rt];
    const V v5 = val[i + dn + lf], v6 = val[i + dn], v7 = val[i + dn + rt];
    const V vi = val[i];
    const V mv = (V)M[i];
    V mm = v0 > v1 ? v0 : v1;
    mm = mm > v2 ? mm : v2;
    mm = mm > v3 ? mm : v3;
    mm = mm > v4 ? mm : v4;
    mm = mm > v5 ? mm : v5;
    mm = mm > v6 ? mm : v6;
    mm = mm > v7 ? mm : v7;
    V nv = mm < mv ? mm : mv;
    if (nv > vi) {
        val[i] = nv;
        return true;
    }
    return false;
}

template <typename L, typename V>
__device__ void recon_scans(const Crop<L> &m, V *val, const int32_t *M) {
    const int lane = threadIdx.x;
    for (;;) {
        bool ch = false;
        for (int r = 0; r < m.ch; ++r) {
            for (int c = lane; c < m.cw; c += blockDim.x) ch |= relax1(m, val, M, r, c);
            __syncthreads();
        }
        for (int r = m.ch - 1; r >= 0; --r) {
            for (int c = lane; c < m.cw; c += blockDim.x) ch |= relax1(m, val, M, r, c);
            __syncthreads();
        }
        for (int c = 0; c < m.cw; ++c) {
            for (int r = lane; r < m.ch; r += blockDim.x) ch |= relax1(m, val, M, r, c);
            __syncthreads();
        }
        for (int c = m.cw - 1; c >= 0; --c) {
            for (int r = lane; r < m.ch; r += blockDim.x) ch |= relax1(m, val, M, r, c);
            __syncthreads();
        }
        if (!wave_or(ch)) break;
    }
}

// ---- reconstruction with the crop in registers (crops of at most R x R) ----
// Same sweeps as recon_scans, but the wave holds the crop as an R x R block
// (lane = column, one register per row), takes the previous row's three
// values from its own register and its neighbours' through DPP wave shifts,
// and transposes through LDS for the horizontal scans.  Pixels outside the
// crop or the component are NEGV in both value and mask, so they neither rise
// nor propagate.
// R = 32: lanes 32..63 mirror lanes 0..31 (same column, same work), so no
// lane is ever masked off; a lane at the crop edge takes NEGV for its outer
// neighbour.
template <int R>
__device__ __forceinline__ bool reg_scan(int (&v)[R], const int (&mk)[R], bool first_col, bool last_col) {
    bool ch = false;
    int pc = NEGV, pl = NEGV, pr = NEGV;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int mm = max(pc, max(pl, pr));
        const int nv = max(v[j], min(mm, mk[j]));
        ch |= nv != v[j];
        v[j] = nv;
        pc = nv;
        const int sl = __builtin_amdgcn_mov_dpp(nv, 0x138, 0xf, 0xf, true);  // lane i <- lane i-1
        const int sr = __builtin_amdgcn_mov_dpp(nv, 0x130, 0xf, 0xf, true);  // lane i <- lane i+1
        pl = first_col ? NEGV : sl;
        pr = last_col ? NEGV : sr;
    }
    pc = pl = pr = NEGV;
#pragma unroll
    for (int j = R - 1; j >= 0; --j) {
        const int mm = max(pc, max(pl, pr));
        const int nv = max(v[j], min(mm, mk[j]));
        ch |= nv != v[j];
        v[j] = nv;
        pc = nv;
        const int sl = __builtin_amdgcn_mov_dpp(nv, 0x138, 0xf, 0xf, true);
        const int sr = __builtin_amdgcn_mov_dpp(nv, 0x130, 0xf, 0xf, true);
        pl = first_col ? NEGV : sl;
        pr = last_col ? NEGV : sr;
    }
    return ch;
}

// In place on the crop plane V, whose row stride is R + 1: the plane is the
// R x (R+1) block the transposes go through.  Entries of V and M outside the
// crop rows and columns, and entries of M outside the component, are set to
// NEGV first (V is NEGV outside the component already; no later step reads
// M there).  Wave 0 holds the registers and runs the sweeps; the other waves
// of the workgroup wait.
template <int R, typename L>
__device__ __forceinline__ void reg_recon(const Crop<L> &m, int32_t *V, int32_t *M) {
    constexpr int TS = R + 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = tid; k < R * TS; k += nt) {
        const int j = k / TS, c = k - j * TS;
        if (j >= m.ch || c >= m.cw) {
            V[k] = NEGV;
            M[k] = NEGV;
        } else if (!(m.fl[k] & F_IN)) {
            M[k] = NEGV;
        }
    }
    __syncthreads();
    if (tid < WAVE) {
        const int cl = tid & (R - 1);
        const bool first = cl == 0, last = cl == R - 1;
        int v[R], mc[R], mr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            v[j] = V[j * TS + cl];
            mc[j] = M[j * TS + cl];
            mr[j] = M[cl * TS + j];
        }
        wave_sync();
        // fixpoint: four consecutive scans (two vertical, two horizontal) that
        // change nothing; V holds the values whenever the loop leaves
        bool hprev = true;   // the previous horizontal scans changed something
        for (;;) {
            const bool cv = __any(reg_scan<R>(v, mc, first, last));
#pragma unroll
            for (int j = 0; j < R; ++j) V[j * TS + cl] = v[j];
            wave_sync();
            if (!cv && !hprev) break;
#pragma unroll
            for (int i = 0; i < R; ++i) v[i] = V[cl * TS + i];
            wave_sync();
            hprev = __any(reg_scan<R>(v, mr, first, last));
#pragma unroll
            for (int i = 0; i < R; ++i) V[cl * TS + i] = v[i];
            wave_sync();
            if (!cv && !hprev) break;
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = V[j * TS + cl];
            wave_sync();
        }
    }
    __syncthreads();
}

// ---- windowed register reconstruction (crops larger than 64 x 64 in LDS) ----
// The crop is covered by 64 x 64 windows at stride 62, so that every pair of
// 8-neighbours lies inside some window.  Each wave takes windows in turn,
// loads one into registers (lane = column), sweeps it to its local fixpoint
// with the scans of reg_recon (through its own 16-bit transpose buffer), and
// raises the plane with an LDS atomic maximum.  Every step only raises values
// towards the result, so windows may overlap and run side by side; passes
// repeat until one changes nothing, and then every neighbour pair satisfies
// the reconstruction's fixpoint condition.
constexpr int WIN = 64, WSTEP = 62, WTS = 65;
constexpr int16_t WNEG = INT16_MIN;   // NEGV in the 16-bit buffers (values here stay far inside int16)

__device__ __forceinline__ int16_t to16(int v) { return v == NEGV ? WNEG : (int16_t)v; }
__device__ __forceinline__ int from16(int16_t v) { return v == WNEG ? NEGV : (int)v; }

template <typename L>
__device__ void win_recon(const Crop<L> &m, int32_t *V, int32_t *M, int16_t *tw, int *flag) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid / WAVE, nwaves = nt / WAVE, lane = tid & (WAVE - 1);
    for (int i = tid; i < m.n; i += nt)
        if (!(m.fl[i] & F_IN)) M[i] = NEGV;   // no later step reads M outside the component
    const int nwx = max(1, (m.cw - 2 + WSTEP - 1) / WSTEP), nwy = max(1, (m.ch - 2 + WSTEP - 1) / WSTEP);
    const int nwin = nwx * nwy;
    int16_t *T = tw + wave * WIN * WTS;
    const bool first = lane == 0, last = lane == WIN - 1;
    for (;;) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int wi = wave; wi < nwin; wi += nwaves) {
            const int wx = (wi % nwx) * WSTEP, wy = (wi / nwx) * WSTEP;
            const int x = wx + lane;
            int v[WIN], mc[WIN], mr[WIN];
#pragma unroll
            for (int j = 0; j < WIN; ++j) {
                const int y = wy + j;
                const bool in = x < m.cw && y < m.ch;
                v[j] = in ? V[y * m.st + x] : NEGV;
                mc[j] = in ? M[y * m.st + x] : NEGV;
                const int yr = wy + lane, xr = wx + j;   // transposed: lane = row
                mr[j] = (yr < m.ch && xr < m.cw) ? M[yr * m.st + xr] : NEGV;
            }
            bool any = false;
            for (;;) {
                bool ch = reg_scan<WIN>(v, mc, first, last);
#pragma unroll
                for (int j = 0; j < WIN; ++j) T[j * WTS + lane] = to16(v[j]);
                wave_sync();
#pragma unroll
                for (int i = 0; i < WIN; ++i) v[i] = from16(T[lane * WTS + i]);
                wave_sync();
                ch |= reg_scan<WIN>(v, mr, first, last);
#pragma unroll
                for (int i = 0; i < WIN; ++i) T[lane * WTS + i] = to16(v[i]);
                wave_sync();
#pragma unroll
                for (int j = 0; j < WIN; ++j) v[j] = from16(T[j * WTS + lane]);
                wave_sync();
                if (!__any(ch)) break;
                any = true;
            }
            if (any) {
#pragma unroll
                for (int j = 0; j < WIN; ++j) {
                    const int y = wy + j;
                    if (x < m.cw && y < m.ch && v[j] != NEGV) atomicMax(V + y * m.st + x, v[j]);
                }
                if (lane == 0) atomicOr(flag, 1);
            }
        }
        __syncthreads();
        const int again = *flag;
        __syncthreads();
        if (!again) break;
    }
}

// V <- recon of V under M: registers when the crop fits R x R; windows of
// registers for the larger LDS crops (tw given); else LDS scans
template <int R, typename L>
__device__ __forceinline__ void recon_any(const Crop<L> &m, int32_t *V, int32_t *M, int16_t *tw = nullptr,
                                          int *flag = nullptr) {
    if constexpr (R > 0) {
        reg_recon<R, L>(m, V, M);
    } else {
        if (tw)
            win_recon<L>(m, V, M, tw, flag);
        else
            recon_scans<L, int32_t>(m, V, M);
    }
}

// ---- one flood level ---------------------------------------------------------
// list[b..e) = the unlabelled pixels of level L.  Keys (distance, label) are
// relaxed from the pixels labelled before L (distance 1) and from pixels of
// the level already reached (distance + 1), in any order, to the fixpoint:
// breadth-first distances with the smallest label at the smallest distance.
template <typename L>
__device__ void flood_level(const Crop<L> &m, const int32_t *list, int b, int e) {
    using K = KeyPack<L>;
    const L one = (L)1 << K::SH;
    const L lmask = one - 1;
    for (;;) {
        bool ch = false;
        for (int pos = b + threadIdx.x; pos < e; pos += blockDim.x) {
            const int i = list[pos];
            const L cur = m.B[i];
            L best = cur <= -2 ? -cur - 2 : (L)-1;  // -1 = none yet (as unsigned compare below)
            const int c = i % m.st, r = i / m.st;
            const int up = r > 0 ? -m.st : 0, dn = r < m.ch - 1 ? m.st : 0;
            const int lf = c > 0 ? -1 : 0, rt = c < m.cw - 1 ? 1 : 0;
            const int nb[8] = {i + up + lf, i + up, i + up + rt, i + lf, i + rt, i + dn + lf, i + dn, i + dn + rt};
            L bv[8];
            uint8_t fv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                bv[k] = m.B[nb[k]];
                fv[k] = m.fl[nb[k]];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // a clamped neighbour is the pixel itself (a current-level pixel:
                // its own key + 1 never beats its key) or a repeated neighbour
                if (!(fv[k] & F_IN)) continue;
                const L bj = bv[k];
                L cand;
                if (bj >= 0)
                    cand = one | bj;
                else if (bj <= -2)
                    cand = (-bj - 2) + one;
                else
                    continue;
                if (best < 0 || cand < best) best = cand;
            }
            if (best >= 0 && (cur > -2 || best < -cur - 2)) {
                m.B[i] = -best - 2;
                ch = true;
            }
        }
        if (!wave_or(ch)) break;
    }
    for (int pos = b + threadIdx.x; pos < e; pos += blockDim.x) {
        const int i = list[pos];
        const L cur = m.B[i];
        if (cur <= -2) m.B[i] = (-cur - 2) & lmask;
    }
    __syncthreads();
}

// number of roots (B[i] == i) of a crop CCL
template <typename L>
__device__ int count_roots(const Crop<L> &m, int *red) {
    int nroots = 0;
    for (int i = threadIdx.x; i < m.n; i += blockDim.x) nroots += (m.B[i] == (L)i);
    if (threadIdx.x == 0) *red = 0;
    __syncthreads();
    if (nroots) atomicAdd(red, nroots);
    __syncthreads();
    const int tot = *red;
    __syncthreads();
    return tot;
}

template <int R>
struct RowMask;
template <>
struct RowMask<32> {
    using T = uint32_t;
};
template <>
struct RowMask<64> {
    using T = uint64_t;
};

// The planes the register-class steps of the distance transform and the
// maxima test use, row stride st: flags, column distances G (capped at 2R)
// and Dq.  The full per-object path keeps G and Dq in 32-bit planes, the
// first small-class pass in bytes (both values stay below 256 there).
template <typename GT, typename DT>
struct RegPlanes {
    const uint8_t *fl;
    GT *G;
    DT *D;
    int st, cw, ch;
};
__device__ __forceinline__ RegPlanes<int32_t, int32_t> reg_planes(const Crop<int32_t> &m) {
    return RegPlanes<int32_t, int32_t>{m.fl, m.A, m.dq, m.st, m.cw, m.ch};
}

// ---- column pass of the distance transform for the register classes ---------
// Crops of at most R rows: thread c < min(cw, R) takes column c and reads its
// membership once into a row mask; the distance of row r to the nearest
// background row above (the highest background bit at or below r) and below
// (the lowest at or above r) come from bit scans, rows at or beyond ch being
// no background (they lie outside the crop).  Stores the column distances
// capped at 2R (the cap the row pass applies; no background in the column:
// the cap).
template <int R, typename GT, typename DT>
__device__ __forceinline__ void edt_cols_reg(const RegPlanes<GT, DT> &m) {
    using MT = typename RowMask<R>::T;
    const int c = threadIdx.x;
    if (c >= R || c >= m.cw) return;
    MT in = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < m.ch && (m.fl[r * m.st + c] & F_IN)) in |= (MT)1 << r;
    const MT rows = m.ch >= R ? ~(MT)0 : (((MT)1 << m.ch) - 1);
    const uint64_t bg = (uint64_t)(~in & rows);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r >= m.ch) break;
        const uint64_t above = r == 63 ? bg : bg & ((2ull << r) - 1);
        const uint64_t below = bg >> r;
        const int up = above ? r - (63 - __builtin_clzll(above)) : 2 * R;
        const int dn = below ? __builtin_ctzll(below) : 2 * R;
        m.G[r * m.st + c] = (GT)min(min(up, dn), 2 * R);
    }
}

// ---- DPP lane shifts of a crop row mask (lane = crop column) ---------------
// Lanes without a source read 0 (bound control), so a row mask shifted in
// from beyond the wave is empty.
__device__ __forceinline__ uint32_t from_left(uint32_t v) {   // lane i <- lane i - 1
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_right(uint32_t v) {  // lane i <- lane i + 1
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ uint64_t from_left(uint64_t v) {
    return (uint64_t)from_left((uint32_t)(v >> 32)) << 32 | from_left((uint32_t)v);
}
__device__ __forceinline__ uint64_t from_right(uint64_t v) {
    return (uint64_t)from_right((uint32_t)(v >> 32)) << 32 | from_right((uint32_t)v);
}
__device__ __forceinline__ int from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }


// ---- regional maxima in registers (register classes) -------------------------
// A component pixel lies in a regional maximum of a plane V iff its plateau
// (the 8-connected set of component pixels of its value through it) has no
// 8-neighbour in the component of larger value: the set V - recon(V - 1
// under V) > 0.  Wave 0 holds one R-bit row mask per column lane (R = 32:
// lanes 32..63 mirror lanes 0..31): it marks the component pixels with a
// larger neighbour, spreads the mark across equal neighbours (vertical steps
// by bit shifts, horizontal and diagonal ones by DPP lane shifts) until it
// stops growing, and returns the unmarked component pixels.  Membership comes
// from the flags; pixels outside the component (and outside the crop rows and
// columns) take NEGV, which no component value reaches, so they are neither
// larger than nor equal to a component pixel.
template <int R, typename GT, typename DT>
__device__ __forceinline__ typename RowMask<R>::T maxima_mask(const RegPlanes<GT, DT> &m) {
    using MT = typename RowMask<R>::T;
    const int c = threadIdx.x & (R - 1);
    const bool first = c == 0, last = c == R - 1, col = c < m.cw;
    MT in = 0, hi = 0, edn = 0, ert = 0, edr = 0, eur = 0;
    auto value = [&](int j) -> int {
        return (col && (m.fl[j * m.st + c] & F_IN)) ? (int)m.D[j * m.st + c] : NEGV;
    };
    // rows j - 1, j, j + 1: own value, left and right neighbours' values
    int dp = NEGV, lp = NEGV, rp = NEGV;
    int dc = value(0);
    int lc = first ? NEGV : from_left(dc), rc = last ? NEGV : from_right(dc);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j >= m.ch) break;
        int dn = NEGV, ln = NEGV, rn = NEGV;
        if (j + 1 < m.ch) {
            dn = value(j + 1);
            ln = first ? NEGV : from_left(dn);
            rn = last ? NEGV : from_right(dn);
        }
        const int mx = max(max(max(dp, dn), max(lc, rc)), max(max(lp, ln), max(rp, rn)));
        const MT bit = (MT)1 << j;
        in |= dc != NEGV ? bit : (MT)0;
        hi |= mx > dc ? bit : (MT)0;
        edn |= dc == dn ? bit : (MT)0;   // (j, c) ~ (j + 1, c)
        ert |= dc == rc ? bit : (MT)0;   // (j, c) ~ (j, c + 1)
        edr |= dc == rn ? bit : (MT)0;   // (j, c) ~ (j + 1, c + 1)
        eur |= dc == rp ? bit : (MT)0;   // (j, c) ~ (j - 1, c + 1)
        dp = dc, lp = lc, rp = rc;
        dc = dn, lc = ln, rc = rn;
    }
    edn &= in, ert &= in, edr &= in, eur &= in;
    MT n = hi & in;   // pixels whose plateau has a larger neighbour
    for (;;) {
        MT nr = from_right(n);
        if (last) nr = 0;
        MT x = (n & ert) | ((n & edr) << 1) | ((n & eur) >> 1);   // what lane c + 1 receives
        MT xl = from_left(x);
        if (first) xl = 0;
        const MT nn = n | ((n & edn) << 1) | ((n >> 1) & edn) | (ert & nr) | (edr & (nr >> 1)) | (eur & (nr << 1)) | xl;
        const bool grew = nn != n;
        n = nn;
        if (!__any(grew)) break;
    }
    return in & ~n;
}

// ---- row-mask set operations of wave 0 (lane = crop column) -----------------
// 8-neighbourhood dilation (the set and its neighbours inside the crop columns
// of the lane layout)
template <int R>
__device__ __forceinline__ typename RowMask<R>::T dilate8(typename RowMask<R>::T f, bool first, bool last) {
    using MT = typename RowMask<R>::T;
    const MT v = f | (f << 1) | (f >> 1);
    MT l = from_left(v), r = from_right(v);
    if (first) l = 0;
    if (last) r = 0;
    return v | l | r;
}
// the first pixel of f in raster order as row * R + column (INT_MAX: f empty)
template <int R>
__device__ __forceinline__ int first_key(typename RowMask<R>::T f, int c) {
    int key = f ? (int)__builtin_ctzll((uint64_t)f) * R + c : INT_MAX;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) key = min(key, __shfl_xor(key, d, WAVE));
    return key;
}
// the 8-connected part of `set` through the pixel `key` (a pixel of set)
template <int R>
__device__ __forceinline__ typename RowMask<R>::T flood_from(typename RowMask<R>::T set, int key, int c, bool first,
                                                             bool last) {
    using MT = typename RowMask<R>::T;
    MT f = (key % R == c) ? (((MT)1 << (key / R)) & set) : (MT)0;
    for (;;) {
        const MT nf = set & dilate8<R>(f, first, last);
        const bool grew = nf != f;
        f = nf;
        if (!__any(grew)) break;
    }
    return f;
}
// number of pixels of f over the crop columns (lanes 0..R-1)
template <int R>
__device__ __forceinline__ int mask_area(typename RowMask<R>::T f) {
    int n = (int)(threadIdx.x & (WAVE - 1)) < R ? __builtin_popcountll((uint64_t)f) : 0;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) n += __shfl_xor(n, d, WAVE);
    return n;
}

// ---- number of regional maxima of Dq, capped at 2 (register classes) --------
// Wave 0 floods from the first maximum pixel in raster order through
// 8-neighbours inside the maxima mask (vertical dilation by bit shifts,
// horizontal by DPP lane shifts) until nothing changes, and reports 0 (no
// maximum), 1 (one 8-connected set) or 2 (a maximum pixel the flood did not
// reach).  Two different regional maxima are never 8-adjacent (the lower of
// two adjacent plateaus has a larger neighbour), so the 8-connected sets of
// the mask are the regional maxima.  The other waves wait.
template <int R, typename L, typename GT, typename DT>
__device__ int count_maxima(const RegPlanes<GT, DT> &m, int *red) {
    using MT = typename RowMask<R>::T;
    const int tid = threadIdx.x;
    if (tid < WAVE) {
        const int c = tid & (R - 1);
        const bool first = c == 0, last = c == R - 1;
        const MT rm = maxima_mask<R>(m);
        int res = 0;
        const int key = first_key<R>(rm, c);
        if (key != INT_MAX) {
            const MT f = flood_from<R>(rm, key, c, first, last);
            res = __any((rm & ~f) != 0) ? 2 : 1;
        }
        if (tid == 0) *red = res;
    }
    crop_sync<L>();
    const int tot = *red;
    crop_sync<L>();
    return tot;
}

__device__ __forceinline__ int isqrt_small(int v) {   // floor(sqrt(v)) for 0 <= v < 2^24
    int r = (int)__builtin_amdgcn_sqrtf((float)v);   // within 1e-3 of sqrt(v): one step each way fixes it
    r -= r * r > v;
    r += (r + 1) * (r + 1) <= v;
    return r;
}

// ---- row pass of the distance transform for the register classes ------------
// Crops of at most R x R in a plane of stride R + 1, NT threads: thread t
// takes row t % R and the output columns c = t / R (mod NH), NH = NT / R.
// With G(c') the column distances the column pass left in A, capped at 2R
// (when the crop holds a background pixel every true distance in it is below
// 2R, so the cap never decides a minimum), the squared distance is
//   min over c' of (c - c')^2 + G(c')^2 = c^2 + min over c' of (E(c') - 2 c' c),
//   E(c') = G(c')^2 + c'^2,
// and E - 2 c' c lies in [-2 * 63 * 63, 128^2 + 63^2] for R <= 64, inside
// 16 bits: two output columns share one packed 16-bit multiply-add and one
// packed minimum per c'.  Columns c' >= cw take E = EPAD, which exceeds every
// candidate of a crop column (at most (2R)^2 - c^2) by more than 2 (R-1)^2,
// so they never decide the minimum and the loop over c' has a fixed length.
typedef short short2_t __attribute__((ext_vector_type(2)));

template <int R, int NT, typename GT, typename DT>
__device__ __forceinline__ void edt_rows_pk(const RegPlanes<GT, DT> &m, bool has_zero) {
    constexpr int NH = NT / R;
    static_assert(NT % R == 0 && R <= 64, "thread layout / 16-bit range");
    const int t = threadIdx.x;
    const int r = t % R, h = t / R, cw = m.cw;
    if (r >= m.ch) return;
    constexpr int EPAD = R == 32 ? 16383 : 32767;
    static_assert(EPAD - 2 * (R - 1) * (R - 1) > 4 * R * R, "padding never decides");
    short2_t e[R / 2];   // E of columns 2k and 2k + 1
#pragma unroll
    for (int cc = 0; cc < R; ++cc) {
        const int gv = min((int)m.G[r * m.st + cc], 2 * R);
        const short ev = cc < cw ? (short)(gv * gv + cc * cc) : (short)EPAD;
        if (cc & 1)
            e[cc / 2].y = ev;
        else
            e[cc / 2].x = ev;
    }
    const int np = (cw + 2 * NH - 1) / (2 * NH);
#pragma unroll 1
    for (int p = 0; p < np; ++p) {
        const int ca = h + 2 * NH * p, cb = ca + NH;
        const short2_t cp = {(short)ca, (short)cb};
        short2_t part[4];   // four independent minimum chains, combined at the end
#pragma unroll
        for (int q = 0; q < 4; ++q) part[q] = short2_t{SHRT_MAX, SHRT_MAX};
#pragma unroll
        for (int cc = 0; cc < R; ++cc) {
            const short2_t k2 = {(short)(-2 * cc), (short)(-2 * cc)};
            const short ev = (cc & 1) ? e[cc / 2].y : e[cc / 2].x;
            const short2_t e2 = {ev, ev};
            part[cc & 3] = __builtin_elementwise_min(part[cc & 3], cp * k2 + e2);
        }
        const short2_t acc = __builtin_elementwise_min(__builtin_elementwise_min(part[0], part[1]),
                                                       __builtin_elementwise_min(part[2], part[3]));
        const int cs[2] = {ca, cb}, bs[2] = {(int)acc.x + ca * ca, (int)acc.y + cb * cb};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = cs[s];
            if (c >= R) continue;
            const int i = r * m.st + c;
            int v = 0;
            if (c < cw && (m.fl[i] & F_IN)) v = has_zero ? isqrt_small(4 * bs[s]) : RT_DQ_MAX;
            m.D[i] = (DT)v;
        }
    }
    if (t < R) m.D[r * m.st + R] = 0;   // the plane's last column (stride R + 1) is padding
}

// ---- seeds, flood, cut and relabelling in registers (register classes) -------
// Entered with g = the h-maxima transform of Dq in plane A; without external
// seeds and seed maps.  The seeds are the regional maxima of g; their
// 8-connected sets, ordered by first pixel (their labels: the crop index of
// that pixel, so label order is raster order), are held by wave 0 as row
// masks S_k.  With more than KMAX of them the call returns -1 and has changed
// nothing (the caller runs the plane-based path); with one it returns 1 (one
// seed: the caller labels the component whole).  Otherwise:
//   * lambda = recon of (Dq on the seeds) under Dq, as in the plane path;
//   * flood, level by level from the highest lambda: the level's unlabelled
//     pixels are reached by synchronous breadth-first steps from the pixels
//     labelled before the level (distance 1) and then from those reached in
//     the previous step; a pixel reached in a step takes the smallest label
//     among the sets that reach it in that step (the smallest key (distance,
//     label) of the plane flood); pixels of a level never reached stay
//     unlabelled;
//   * cut: a labelled pixel is kept iff no component neighbour has a smaller
//     label or is unlabelled (unlabelled pixels count as label -1 and are
//     always kept), so the kept pixels of different labels are never adjacent;
//   * relabelling: each 8-connected piece of the kept pixels of one label (or
//     of the unlabelled ones) is labelled by its first pixel and kept when
//     its area passes the final filter; the component's pixels are written.
// Returns 2 when the component is done.  The seed sets wait in plane B (as
// 64-bit words) while the lambda reconstruction holds the registers.
constexpr int KMAX = 8;

template <int R, typename L>
__device__ int reg_watershed(const ObjArgs &a, const Crop<L> &m, int *red, int16_t *tw) {
    using MT = typename RowMask<R>::T;
    const int tid = threadIdx.x;
    const int c = tid & (R - 1);
    const bool first = c == 0, last = c == R - 1, lead = tid < WAVE;
    const bool col = c < m.cw, writer = tid < R && col;
    uint64_t *stash = (uint64_t *)m.B;   // KMAX x WAVE words (plane B holds at least R (R + 1) 4-byte entries)
    MT S[KMAX];
    int K = 0;
    if (lead) {
        const MT rm = maxima_mask<R>(RegPlanes<int32_t, int32_t>{m.fl, m.A, m.A, m.st, m.cw, m.ch});
        MT rest = rm;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            S[k] = 0;
            if (__any(rest != 0)) {
                S[k] = flood_from<R>(rest, first_key<R>(rest, c), c, first, last);
                rest &= ~S[k];
                ++K;
            }
        }
        if (__any(rest != 0)) K = KMAX + 1;
        if (tid == 0) *red = K;
    }
    crop_sync<L>();
    K = *red;
    crop_sync<L>();
    if (K > KMAX) return -1;
    if (K <= 1) return 1;
    // lambda marker: Dq on the seeds (wave 0 writes its columns; reg_recon
    // sets everything outside the crop and the component itself)
    if (lead) {
        MT seeds = 0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            seeds |= S[k];
            stash[k * WAVE + tid] = (uint64_t)S[k];
        }
        if (writer)
            for (int j = 0; j < m.ch; ++j) {
                const int i = j * m.st + c;
                m.A[i] = ((seeds >> j) & 1) ? m.dq[i] : NEGV;
            }
    }
    crop_sync<L>();
    recon_any<R, L>(m, m.A, m.dq, tw, red);   // A = lambda
    int kept = 0;
    if (lead) {
        // lambda of the component's pixels as eight bit planes (lambda lies
        // between the smallest and the largest Dq of the component, and Dq of a
        // crop of at most 64 x 64 that holds a background pixel is below
        // 2 * 64 * sqrt(2) < 256)
        MT inm = 0, lab = 0, bp[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) bp[b] = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (j < m.ch && col && (m.fl[j * m.st + c] & F_IN)) {
                inm |= (MT)1 << j;
                const unsigned v = (unsigned)m.A[j * m.st + c];
#pragma unroll
                for (int b = 0; b < 8; ++b) bp[b] |= (MT)((v >> b) & 1u) << j;
            }
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            S[k] = (MT)stash[k * WAVE + tid];
            lab |= S[k];
        }
        MT U = inm & ~lab, unreached = 0;
        // flood, level by level; the pixels of U at the highest lambda come
        // from the bit planes, top bit first (keep the candidates that have the
        // bit whenever some do)
        while (__any(U != 0)) {
            MT lv = U;
#pragma unroll
            for (int b = 7; b >= 0; --b) {
                const MT t = lv & bp[b];
                if (__any(t != 0)) lv = t;
            }
            U &= ~lv;
            MT F[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) F[k] = S[k];
            for (;;) {
                MT taken = 0;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < K) {   // K is uniform: a scalar branch
                        const MT nk = dilate8<R>(F[k], first, last) & lv & ~taken;
                        taken |= nk;
                        F[k] = nk;
                        S[k] |= nk;
                    }
                }
                lv &= ~taken;
                if (!__any(taken != 0)) break;
            }
            unreached |= lv;
        }
        unreached |= U;   // pixels lambda never reached (none when every pixel is connected to a seed)
        // cut: kept iff no neighbour of a smaller label (unreached pixels: -1)
        MT P = unreached, keep_all = unreached;
        MT keep[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            keep[k] = 0;
            if (k < K) {
                keep[k] = S[k] & ~dilate8<R>(P, first, last);
                P |= S[k];
                keep_all |= keep[k];
            }
        }
        // pixels cut away
        const int64_t rowbase = (int64_t)m.cy0 * a.pitch + m.cx0 + c;
        if (writer)
            for (MT b = inm & ~keep_all; b; b &= b - 1) {
                const int64_t o = rowbase + (int64_t)__builtin_ctzll((uint64_t)b) * a.pitch;
                a.labels[o] = 0;
                a.mask[o] = 0;
            }
        // pieces of each label's kept pixels, and of the unreached ones
#pragma unroll
        for (int k = 0; k <= KMAX; ++k) {
            if (k < KMAX && k >= K) continue;
            MT rest = k < KMAX ? keep[k] : unreached;
            while (__any(rest != 0)) {
                const int key = first_key<R>(rest, c);
                const MT f = flood_from<R>(rest, key, c, first, last);
                rest &= ~f;
                const int ar = mask_area<R>(f);
                int lb = 0;
                if (ar >= a.min_area && (a.max_area < 0 || ar <= a.max_area)) {
                    lb = (m.cy0 + key / R) * a.w + m.cx0 + key % R + 1;
                    ++kept;
                }
                if (writer)
                    for (MT b = f; b; b &= b - 1) {
                        const int64_t o = rowbase + (int64_t)__builtin_ctzll((uint64_t)b) * a.pitch;
                        a.labels[o] = lb;
                        a.mask[o] = lb ? 1 : 0;
                    }
            }
        }
        if (tid == 0 && kept && a.n_kept) atomicAdd(a.n_kept, kept);
    }
    crop_sync<L>();
    return 2;
}

// ---- the whole per-component stage ---------------------------------------------
template <int R, typename L>
__device__ __forceinline__ void process_object(const ObjArgs &a, int g, Crop<L> m, int *red, int *hist, int16_t *tw = nullptr) {
    const int lane = threadIdx.x;
    const int area = a.st_area[g];
    // ---- load the component: LOADS_IN_FLIGHT loads per thread issued before
    // any is used (addresses clamped into the crop, crop_addr.h)
    const CropGeom geom{m.cx0, m.cy0, m.cw, m.ch, m.st, m.n};
    bool zero = false;
    if constexpr (R == RS_ || R == RM_) {
        // register classes: loads by crop pixel (no padding column), the flag
        // plane cleared (32-bit stores; the plane capacity is a multiple of 4)
        // while the first batch is in flight
        const int npx = m.cw * m.ch, nt = blockDim.x;
        const float inv_cw = 1.0f / (float)m.cw;
        for (int k0 = 0; k0 < npx; k0 += LOADS_IN_FLIGHT * nt) {
            int32_t v[LOADS_IN_FLIGHT];
#pragma unroll
            for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
                v[k] = a.labels[crop_load_offset_dense(geom, k0 + k * nt + lane, inv_cw, a.pitch)];
            if (k0 == 0) {
                for (int w = lane; w < (m.n + 3) / 4; w += nt) ((uint32_t *)m.fl)[w] = 0;
                crop_sync<L>();
            }
#pragma unroll
            for (int k = 0; k < LOADS_IN_FLIGHT; ++k) {
                const int kk = k0 + k * nt + lane;
                if (kk < npx) {
                    const int r = crop_dense_row(kk, inv_cw);
                    const bool in = v[k] == g;
                    zero |= !in;
                    if (in) m.fl[r * m.st + kk - r * m.cw] = F_IN;
                }
            }
        }
    } else {
        for (int i0 = 0; i0 < m.n; i0 += LOADS_IN_FLIGHT * (int)blockDim.x) {
            int32_t v[LOADS_IN_FLIGHT];
#pragma unroll
            for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
                v[k] = a.labels[crop_load_offset(geom, i0 + k * (int)blockDim.x + lane, a.pitch)];
#pragma unroll
            for (int k = 0; k < LOADS_IN_FLIGHT; ++k) {
                const int i = i0 + k * (int)blockDim.x + lane;
                if (i < m.n) {
                    const bool col = i % m.st < m.cw;
                    const bool in = col && v[k] == g;
                    zero |= col && !in;
                    m.fl[i] = in ? F_IN : 0;
                }
            }
        }
    }
    const bool has_zero = crop_any<L>(zero);
    // ---- exact distance transform: column distances, then the row pass
    if constexpr (R == RS_ || R == RM_) {
        edt_cols_reg<R>(reg_planes(m));
    } else {
        for (int c = lane; c < m.cw; c += blockDim.x) {
            int run = GINF;
            for (int r = 0; r < m.ch; ++r) {
                const int i = r * m.st + c;
                run = (m.fl[i] & F_IN) ? (run < GINF ? run + 1 : GINF) : 0;
                m.A[i] = run;
            }
            run = GINF;
            for (int r = m.ch - 1; r >= 0; --r) {
                const int i = r * m.st + c;
                run = (m.fl[i] & F_IN) ? (run < GINF ? run + 1 : GINF) : 0;
                if (run < m.A[i]) m.A[i] = run;
            }
        }
    }
    crop_sync<L>();
    if constexpr (R == RS_) {
        edt_rows_pk<RS_, WAVE>(reg_planes(m), has_zero);
    } else if constexpr (R == RM_) {
        edt_rows_pk<RM_, 2 * WAVE>(reg_planes(m), has_zero);
    } else {
        for (int i = lane; i < m.n; i += blockDim.x) {
            const int c = i % m.st, r = i / m.st;
            if (c >= m.cw || !(m.fl[i] & F_IN)) {
                m.dq[i] = 0;
                continue;
            }
            if (!has_zero) {  // the crop is the whole tile and all foreground
                m.dq[i] = RT_DQ_MAX;
                continue;
            }
            const int32_t *row = m.A + r * m.st;
            int64_t best = row[c] < GINF ? (int64_t)row[c] * row[c] : INT64_MAX;
            for (int dx = 1;; ++dx) {
                const int64_t dd = (int64_t)dx * dx;
                if (dd >= best) break;
                const bool lo = c - dx >= 0, hi = c + dx < m.cw;
                if (!lo && !hi) break;
                if (lo && row[c - dx] < GINF) best = min(best, dd + (int64_t)row[c - dx] * row[c - dx]);
                if (hi && row[c + dx] < GINF) best = min(best, dd + (int64_t)row[c + dx] * row[c + dx]);
            }
            m.dq[i] = isqrt_exact(4 * best);
        }
    }
    crop_sync<L>();
    int tot = 0;
    bool one_seed = false;   // the register path found one seed
    {
        // ---- seeds
        if (a.seeds) {
            for (int i0 = 0; i0 < m.n; i0 += LOADS_IN_FLIGHT * (int)blockDim.x) {
                uint8_t v[LOADS_IN_FLIGHT];
#pragma unroll
                for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
                    v[k] = a.seeds[crop_load_offset(geom, i0 + k * (int)blockDim.x + lane, a.pitch)];
#pragma unroll
                for (int k = 0; k < LOADS_IN_FLIGHT; ++k) {
                    const int i = i0 + k * (int)blockDim.x + lane;
                    if (i < m.n && (m.fl[i] & F_IN) && v[k]) m.fl[i] |= F_RM;
                }
            }
            __syncthreads();
        } else {
            for (int i = lane; i < m.n; i += blockDim.x) m.A[i] = (m.fl[i] & F_IN) ? m.dq[i] - a.h_seed : NEGV;
            __syncthreads();
            recon_any<R, L>(m, m.A, m.dq, tw, red);  // g = h-maxima of Dq
            if constexpr (R == RS_ || R == RM_) {
                if (!a.fg_out) {
                    const int r = reg_watershed<R, L>(a, m, red, tw);
                    if (r == 2) return;
                    one_seed = r == 1;
                }
            }
            if (!one_seed) {
                for (int i = lane; i < m.n; i += blockDim.x) m.B[i] = (m.fl[i] & F_IN) ? (L)(m.A[i] - 1) : (L)NEGV;
                __syncthreads();
                if constexpr (R > 0 || sizeof(L) == 4)
                    recon_any<R, L>(m, (int32_t *)m.B, m.A, tw, red);   // recon of g-1 under g
                else
                    recon_scans<L, L>(m, m.B, m.A);
                for (int i = lane; i < m.n; i += blockDim.x)
                    if ((m.fl[i] & F_IN) && (L)m.A[i] - m.B[i] > 0) m.fl[i] |= F_RM;
                __syncthreads();
            }
        }
        if (one_seed) {
            tot = 1;
        } else {
            if (a.fg_out) {   // the foreground A and its seed map, for callers that want them
                for (int i = lane; i < m.n; i += blockDim.x) {
                    if (!(m.fl[i] & F_IN)) continue;
                    const int c = i % m.st, r = i / m.st;
                    const int64_t o = (int64_t)(m.cy0 + r) * a.pitch + m.cx0 + c;
                    a.fg_out[o] = 1;
                    a.seeds_out[o] = (m.fl[i] & F_RM) ? 1 : 0;
                }
            }
            crop_ccl<L, L>(m, F_RM, m.B);  // B = seed label (crop index of the seed root) or -1
            tot = count_roots(m, red);
        }
    }
    const bool area_ok = area >= a.min_area && (a.max_area < 0 || area <= a.max_area);
    if (tot <= 1) {
        // one seed (or none with external seeds): the whole component gets one
        // label, nothing is cut, and the relabelled component is the component
        // (its pixels already hold the label g)
        if constexpr (R == RS_ || R == RM_) {
            const int npx = m.cw * m.ch;
            const float inv_cw = 1.0f / (float)m.cw;
            for (int k = lane; k < npx; k += blockDim.x) {
                const int r = crop_dense_row(k, inv_cw), c = k - r * m.cw;
                if (!(m.fl[r * m.st + c] & F_IN)) continue;
                const int64_t o = (int64_t)(m.cy0 + r) * a.pitch + m.cx0 + c;
                if (!area_ok) a.labels[o] = 0;
                a.mask[o] = area_ok ? 1 : 0;
            }
        } else {
            for (int i = lane; i < m.n; i += blockDim.x) {
                if (!(m.fl[i] & F_IN)) continue;
                const int c = i % m.st, r = i / m.st;
                const int64_t o = (int64_t)(m.cy0 + r) * a.pitch + m.cx0 + c;
                if (!area_ok) a.labels[o] = 0;
                a.mask[o] = area_ok ? 1 : 0;
            }
        }
        if (lane == 0 && area_ok && a.n_kept) atomicAdd(a.n_kept, 1);
        crop_sync<L>();
        return;
    }
    // ---- lambda = recon of (Dq on seeds) under Dq
    for (int i = lane; i < m.n; i += blockDim.x) m.A[i] = ((m.fl[i] & F_IN) && (m.fl[i] & F_RM)) ? m.dq[i] : NEGV;
    __syncthreads();
    recon_any<R, L>(m, m.A, m.dq, tw, red);
    // ---- flood, level by level from the highest lambda
    int lmax = NEGV, lmin = INT_MAX;
    for (int i = lane; i < m.n; i += blockDim.x)
        if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] != NEGV) {
            lmax = max(lmax, m.A[i]);
            lmin = min(lmin, m.A[i]);
        }
    lmax = wave_max(lmax, red);
    lmin = wave_min(lmin, red);
    int32_t *list = m.dq;  // Dq is no longer needed
    if (lmax != NEGV) {
        const int range = lmax - lmin + 1;
        if (range <= HBINS) {
            // counting sort of the unlabelled pixels by decreasing lambda
            for (int k = lane; k <= HBINS; k += blockDim.x) hist[k] = 0;
            __syncthreads();
            for (int i = lane; i < m.n; i += blockDim.x)
                if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] != NEGV) atomicAdd(hist + 1 + (lmax - m.A[i]), 1);
            __syncthreads();
            if (lane == 0)
                for (int k = 1; k <= HBINS; ++k) hist[k] += hist[k - 1];
            __syncthreads();
            // hist[k] = start of bin k; scatter with a moving cursor per bin
            for (int i = lane; i < m.n; i += blockDim.x)
                if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] != NEGV) {
                    const int pos = atomicAdd(hist + (lmax - m.A[i]), 1);
                    list[pos] = i;
                }
            __syncthreads();
            // after the scatter hist[k] = end of bin k
            int b = 0;
            for (int k = 0; k < range; ++k) {
                const int e = hist[k];
                if (e > b) flood_level<L>(m, list, b, e);
                b = e;
            }
        } else {
            // wide range: find each level, compact its pixels, flood it
            for (int L0 = lmax; L0 != NEGV;) {
                if (lane == 0) *red = 0;
                __syncthreads();
                for (int i = lane; i < m.n; i += blockDim.x)
                    if ((m.fl[i] & F_IN) && m.B[i] == -1 && m.A[i] == L0) list[atomicAdd(red, 1)] = i;
                __syncthreads();
                const int cnt = *red;
                __syncthreads();
                flood_level<L>(m, list, 0, cnt);
                int nxt = NEGV;
                for (int i = lane; i < m.n; i += blockDim.x)
                    if ((m.fl[i] & F_IN) && m.B[i] < 0 && m.A[i] != NEGV && m.A[i] < L0) nxt = max(nxt, m.A[i]);
                L0 = wave_max(nxt, red);
            }
        }
    }
    // ---- leftovers (external seeds only): their own components
    if (a.seeds) {
        bool left = false;
        for (int i = lane; i < m.n; i += blockDim.x)
            if ((m.fl[i] & F_IN) && m.B[i] < 0) {
                m.fl[i] |= F_M;
                left = true;
            }
        if (wave_or(left)) {
            crop_ccl<L, int32_t>(m, F_M, m.A);
            for (int i = lane; i < m.n; i += blockDim.x)
                if (m.fl[i] & F_M) m.B[i] = m.A[i];
            __syncthreads();
        }
        for (int i = lane; i < m.n; i += blockDim.x) m.fl[i] &= (uint8_t)~F_M;
        __syncthreads();
    }
    // ---- cut: keep p iff no neighbour in the component has a smaller label
    for (int i = lane; i < m.n; i += blockDim.x) {
        if (!(m.fl[i] & F_IN)) continue;
        const int c = i % m.st, r = i / m.st;
        const L lab = m.B[i];
        const int up = r > 0 ? -m.st : 0, dn = r < m.ch - 1 ? m.st : 0;
        const int lf = c > 0 ? -1 : 0, rt = c < m.cw - 1 ? 1 : 0;
        const int nb[8] = {i + up + lf, i + up, i + up + rt, i + lf, i + rt, i + dn + lf, i + dn, i + dn + rt};
        bool keep = true;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((m.fl[nb[k]] & F_IN) && m.B[nb[k]] < lab) keep = false;
        if (keep) m.fl[i] |= F_M;
    }
    __syncthreads();
    // ---- relabel the kept pixels, area of each piece, write out
    crop_ccl<L, int32_t>(m, F_M, m.A);
    int32_t *cnt = m.dq;
    for (int i = lane; i < m.n; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    for (int i = lane; i < m.n; i += blockDim.x)
        if (m.fl[i] & F_M) atomicAdd(cnt + m.A[i], 1);
    __syncthreads();
    int kept = 0;
    for (int i = lane; i < m.n; i += blockDim.x) {
        if (!(m.fl[i] & F_IN)) continue;
        const int c = i % m.st, r = i / m.st;
        const int64_t o = (int64_t)(m.cy0 + r) * a.pitch + m.cx0 + c;
        int lab = 0;
        if (m.fl[i] & F_M) {
            const int root = m.A[i];
            const int ar = cnt[root];
            if (ar >= a.min_area && (a.max_area < 0 || ar <= a.max_area)) {
                lab = (m.cy0 + root / m.st) * a.w + m.cx0 + root % m.st + 1;
                if (root == i) ++kept;
            }
        }
        a.labels[o] = lab;
        a.mask[o] = lab ? 1 : 0;
    }
    if (a.n_kept && kept) atomicAdd(a.n_kept, kept);
    __syncthreads();
}

__device__ __forceinline__ CropGeom crop_geom(const ObjArgs &a, int g) {
    return crop_of_box(a.st_x0[g], a.st_y0[g], a.st_x1[g], a.st_y1[g], a.w, a.h);
}

// The register classes use the row stride R + 1 of the in-place register
// reconstruction (the plane capacity is R x (R + 1)).
__device__ __forceinline__ CropGeom with_stride(CropGeom q, int st) { return crop_with_stride(q, st); }

// One wave per component: lane = crop column (strips of 64 columns), eight
// rows' loads issued before any is tested.
__device__ void erase_object(const ObjArgs &a, int g, const CropGeom &q) {
    for (int c = threadIdx.x; c < q.cw; c += WAVE)
        for (int r0 = 0; r0 < q.ch; r0 += 8) {
            int32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = a.labels[crop_erase_offset(q, c, r0 + k, a.pitch)];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (r0 + k < q.ch && v[k] == g) {
                    const int64_t o = crop_erase_offset(q, c, r0 + k, a.pitch);
                    a.labels[o] = 0;
                    a.mask[o] = 0;
                }
        }
}

// ---- first small-class pass: components with at most one seed ---------------
// Crops of at most 32 x 32, one wave, byte planes (flags, capped column
// distances, Dq: all below 256 for these crops) in `pl` (3 CAP_S bytes), so
// many waves fit a CU.  Loads the component, and unless its crop holds no
// background pixel (then Dq is constant on it: one maximum), runs the
// distance transform and counts the regional maxima of Dq.  At most one
// means one seed: each regional maximum of the h-maxima transform
// g = recon(Dq - h under Dq) contains a regional maximum of Dq (a plateau of g
// at value v holds a point with Dq - h = v, and the component of
// {Dq >= v + h} through it stays inside the plateau, so its top is a regional
// maximum of Dq), so g has at most as many.  Then the component keeps its
// label g when its area passes the final filter and is erased otherwise, and
// the call returns true.  Otherwise it returns false and writes nothing: the
// caller defers the component to the full path.
__device__ __forceinline__ bool single_seed_object(const ObjArgs &a, int g, const CropGeom &q, uint8_t *pl, int *red) {
    const int lane = threadIdx.x;
    const RegPlanes<uint8_t, uint8_t> p{pl, pl + CAP_S, pl + 2 * CAP_S, q.st, q.cw, q.ch};
    uint8_t *fl = pl;
    const int npx = q.cw * q.ch;
    const float inv_cw = 1.0f / (float)q.cw;
    bool zero = false;
    for (int k0 = 0; k0 < npx; k0 += LOADS_IN_FLIGHT * WAVE) {
        int32_t v[LOADS_IN_FLIGHT];
#pragma unroll
        for (int k = 0; k < LOADS_IN_FLIGHT; ++k)
            v[k] = a.labels[crop_load_offset_dense(q, k0 + k * WAVE + lane, inv_cw, a.pitch)];
        if (k0 == 0)
            for (int w = lane; w < (q.n + 3) / 4; w += WAVE) ((uint32_t *)fl)[w] = 0;
        wave_sync();
#pragma unroll
        for (int k = 0; k < LOADS_IN_FLIGHT; ++k) {
            const int kk = k0 + k * WAVE + lane;
            if (kk < npx) {
                const int r = crop_dense_row(kk, inv_cw);
                const bool in = v[k] == g;
                zero |= !in;
                if (in) fl[r * q.st + kk - r * q.cw] = F_IN;
            }
        }
    }
    wave_sync();
    int tot = 1;
    if (__any(zero)) {
        edt_cols_reg<RS_>(p);
        wave_sync();
        edt_rows_pk<RS_, WAVE>(p, true);
        wave_sync();
        tot = count_maxima<RS_, int32_t>(p, red);
    }
    if (tot > 1) return false;
    const int area = a.st_area[g];
    const bool area_ok = area >= a.min_area && (a.max_area < 0 || area <= a.max_area);
    for (int k = lane; k < npx; k += WAVE) {
        const int r = crop_dense_row(k, inv_cw), c = k - r * q.cw;
        if (!(fl[r * q.st + c] & F_IN)) continue;
        const int64_t o = (int64_t)(q.cy0 + r) * a.pitch + q.cx0 + c;
        if (!area_ok) a.labels[o] = 0;
        a.mask[o] = area_ok ? 1 : 0;
    }
    if (lane == 0 && area_ok && a.n_kept) atomicAdd(a.n_kept, 1);
    wave_sync();
    return true;
}

template <int CAP>
__device__ __forceinline__ Crop<int32_t> lds_crop(unsigned char *smem, const CropGeom &q) {
    Crop<int32_t> m;
    m.dq = (int32_t *)smem;
    m.A = m.dq + CAP;
    m.B = m.A + CAP;
    m.fl = (uint8_t *)(m.B + CAP);
    m.st = q.st;
    m.cw = q.cw;
    m.ch = q.ch;
    m.cx0 = q.cx0;
    m.cy0 = q.cy0;
    m.n = q.n;
    return m;
}

constexpr int CODE_MASK = (1 << 25) - 1;   // component code = image << 25 | root

// Routes every registered component to its class list (one thread per
// component, appends aggregated per wave): components below the first area
// threshold and crops up to 32 x 32 to the small class (which erases the
// former), up to 64 x 64 to the medium class, up to CAP_L pixels to the large
// LDS class, the rest to global memory.
__device__ __forceinline__ void wave_append(bool want, int code, int32_t *list, int32_t *cnt) {
    const uint64_t m = __ballot(want);
    if (!m) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int leader = __builtin_ctzll(m);
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt, __popcll(m));
    base = __shfl(base, leader, WAVE);
    if (want) list[base + __popcll(m & ((1ull << lane) - 1))] = code;
}

__global__ void k_objects_classify(const ObjArgs *args, ObjLists L) {
    const int nobj = *L.n_obj;
    const int stride = gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations (ballots)
    const int iters = (nobj + stride - 1) / stride;
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    for (int it = 0; it < iters; ++it, o += stride) {
        int cls = -1, code = 0;
        if (o < nobj) {
            code = L.obj[o];
            const ObjArgs a = args[code >> 25];
            const int g = code & CODE_MASK;
            const CropGeom q = crop_geom(a, g);
            if (a.st_area[g] < a.min_area_pre)
                cls = 4;
            else if (L.path != 2 && q.cw <= RS_ && q.ch <= RS_)
                cls = 0;
            else if (L.path == 0 && q.cw <= RM_ && q.ch <= RM_)
                cls = 1;
            else if (q.n <= CAP_L)
                cls = 2;
            else
                cls = 3;
        }
        wave_append(cls == 0, code, L.list_s, L.n_s);
        wave_append(cls == 1, code, L.list_m, L.n_m);
        wave_append(cls == 2, code, L.list_l, L.n_l);
        wave_append(cls == 3, code, L.big, L.n_big);
        wave_append(cls == 4, code, L.list_e, L.n_e);
    }
}

// components below the first area threshold: their pixels are cleared in
// the labels and the mask (one wave each)
__global__ __launch_bounds__(WAVE) void k_objects_erase(const ObjArgs *args, ObjLists L) {
    const int nobj = *L.n_e;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int code = L.list_e[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        erase_object(a, g, crop_geom(a, g));
    }
}

// small class, first pass: finishes the crops up to 32 x 32 with at most one
// seed, and defers the others (and, with external seeds or seed maps wanted,
// every component) to the full pass
__global__ __launch_bounds__(WAVE, 6) void k_objects_s1(const ObjArgs *args, ObjLists L) {
    __shared__ __align__(16) uint8_t pl[3 * CAP_S];
    __shared__ int red;
    const int nobj = *L.n_s;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int code = L.list_s[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        const CropGeom q = crop_geom(a, g);
        const bool done = !a.seeds && !a.fg_out && single_seed_object(a, g, with_stride(q, RS_ + 1), pl, &red);
        if (!done && threadIdx.x == 0) L.list_sd[atomicAdd(L.n_sd, 1)] = code;
    }
}

// small class, full pass: the deferred components, crops up to 32 x 32
__global__ __launch_bounds__(WAVE, 2) void k_objects_s(const ObjArgs *args, ObjLists L) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int red;
    __shared__ int hist[HBINS + 1];
    const int nobj = *L.n_sd;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int code = L.list_sd[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        process_object<RS_, int32_t>(a, g, lds_crop<CAP_S>(smem, with_stride(crop_geom(a, g), RS_ + 1)), &red, hist);
    }
}

__global__ __launch_bounds__(2 * WAVE) void k_objects_m(const ObjArgs *args, ObjLists L) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int red;
    __shared__ int hist[HBINS + 1];
    const int nobj = *L.n_m;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int code = L.list_m[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        const CropGeom q = crop_geom(a, g);
        if (q.cw > RM_ || q.ch > RM_) {   // routed here only when it fits; the global class takes any crop
            if (threadIdx.x == 0) L.big[atomicAdd(L.n_big, 1)] = code;
            continue;
        }
        process_object<RM_, int32_t>(a, g, lds_crop<CAP_M>(smem, with_stride(q, RM_ + 1)), &red, hist);
    }
}

// large class: crops up to CAP_L pixels in LDS, scans without the register
// path (one workgroup per CU for LDS); four waves per component, so a row
// of the directional scans is one pass
__global__ __launch_bounds__(4 * WAVE) void k_objects_l(const ObjArgs *args, ObjLists L) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int red;
    __shared__ int hist[HBINS + 1];
    const int nobj = *L.n_l;
    for (int o = blockIdx.x; o < nobj; o += gridDim.x) {
        const int code = L.list_l[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        const CropGeom q = crop_geom(a, g);
        if (q.n > CAP_L) {   // routed here only when it fits; keep the guard for the LDS bound
            if (threadIdx.x == 0) L.big[atomicAdd(L.n_big, 1)] = code;
            continue;
        }
        process_object<0, int32_t>(a, g, lds_crop<CAP_L>(smem, q), &red, hist,
                                   (int16_t *)(smem + (size_t)CAP_L * 13));
    }
}

// global-memory class: one wave per component on a scratch slice.  Two
// passes: crops up to mid_max_px on many moderate slices, deferring larger
// ones to a second pass on a few slices sized for the whole tile.
struct BigPass {
    const int32_t *list, *n;
    int32_t *defer, *n_defer;   // nullable
    char *scratch;
    size_t slice_bytes;
    int64_t max_px;             // crops above this are deferred (when defer is set)
};

__global__ __launch_bounds__(WAVE) void k_objects_big(const ObjArgs *args, BigPass P) {
    __shared__ int red;
    __shared__ int hist[HBINS + 1];
    const int nbig = *P.n;
    char *base = P.scratch + P.slice_bytes * blockIdx.x;
    for (int o = blockIdx.x; o < nbig; o += gridDim.x) {
        const int code = P.list[o];
        const ObjArgs a = args[code >> 25];
        const int g = code & CODE_MASK;
        const CropGeom q = crop_geom(a, g);
        if (P.defer && (int64_t)q.n > P.max_px) {
            if (threadIdx.x == 0) P.defer[atomicAdd(P.n_defer, 1)] = code;
            continue;
        }
        Crop<int64_t> m;
        m.B = (int64_t *)base;
        m.dq = (int32_t *)(m.B + q.n);
        m.A = m.dq + q.n;
        m.fl = (uint8_t *)(m.A + q.n);
        m.st = q.st;
        m.cw = q.cw;
        m.ch = q.ch;
        m.cx0 = q.cx0;
        m.cy0 = q.cy0;
        m.n = q.n;
        process_object<0, int64_t>(a, g, m, &red, hist);
    }
}

// Profiling tally: pixels of the components each LDS class took (sum of the
// component areas over the class lists), summed by a grid-stride pass after
// the per-object stage; the class kernels themselves are not instrumented.
__global__ __launch_bounds__(256) void k_objects_tally(const ObjArgs *args, ObjLists L, unsigned long long *out) {
    __shared__ unsigned long long part[3];
    if (threadIdx.x < 3) part[threadIdx.x] = 0;
    __syncthreads();
    const int32_t *lists[3] = {L.list_s, L.list_m, L.list_l};
    const int32_t *counts[3] = {L.n_s, L.n_m, L.n_l};
    for (int k = 0; k < 3; ++k) {
        const int n = *counts[k];
        unsigned long long s = 0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const int code = lists[k][i];
            s += (unsigned long long)args[code >> 25].st_area[code & CODE_MASK];
        }
        if (s) atomicAdd(part + k, s);
    }
    __syncthreads();
    if (threadIdx.x < 3 && part[threadIdx.x]) atomicAdd(out + threadIdx.x, part[threadIdx.x]);
}

int launch_objects_tally(const ObjArgs *args_dev, const ObjLists &L, unsigned long long *out, int n_cu,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_objects_tally, dim3(n_cu), dim3(256), 0, s, args_dev, L, out);
    return hip_fail(hipGetLastError(), "k_objects_tally");
}

// bytes of global scratch one block needs for a crop of n = stride x rows pixels
static size_t crop_bytes(int64_t n) { return (size_t)n * (8 + 4 + 4 + 1) + 256; }
// ... and for the largest crop of a w x h tile
size_t big_object_bytes(int w, int h) { return crop_bytes((int64_t)h * (w | 1)); }
size_t mid_object_bytes(int w, int h) { return std::min(big_object_bytes(w, h), crop_bytes(MID_MAX_PX)); }

int launch_objects(const ObjArgs *args_dev, const ObjLists &L, int n_cu, hipStream_t s, hipEvent_t before_big,
                   const ObjStreams *par) {
    if (L.big_slices < 1 || L.mid_slices < 1) {
        set_error("objects: no global scratch slice");
        return RT_ENOMEM;
    }
    const size_t lds_s = (size_t)CAP_S * 13, lds_m = (size_t)CAP_M * 13;
    const size_t lds_l = (size_t)CAP_L * 13 + 4 * WIN * WTS * sizeof(int16_t);   // planes + 4 window buffers
    static bool lds_l_set = false;
    if (!lds_l_set) {
        RT_HIP(hipFuncSetAttribute((const void *)k_objects_l, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_l));
        lds_l_set = true;
    }
    hipLaunchKernelGGL(k_objects_classify, dim3(n_cu * 4), dim3(256), 0, s, args_dev, L);
    RT_HIP(hipGetLastError());
    // With side streams the three LDS classes run side by side: the medium
    // class on the caller's stream, the small class and the large class on
    // one side stream each (a large component is the longest single piece
    // of work, the many small ones fill the compute units around it).
    hipStream_t t = s, u = s;
    if (par && par->side && par->side2) {
        RT_HIP(hipEventRecord(par->fork, s));
        RT_HIP(hipStreamWaitEvent(par->side, par->fork, 0));
        RT_HIP(hipStreamWaitEvent(par->side2, par->fork, 0));
        t = par->side;
        u = par->side2;
    }
    // class timing (profiling): an event pair around each launch on its own stream
    auto mark = [&](int cls, int end, hipStream_t st) -> int {
        if (par && par->timing[cls][end]) RT_HIP(hipEventRecord(par->timing[cls][end], st));
        return RT_OK;
    };
    int e;
    hipLaunchKernelGGL(k_objects_erase, dim3(n_cu * 8), dim3(WAVE), 0, u, args_dev, L);
    RT_HIP(hipGetLastError());
    if ((e = mark(2, 0, u))) return e;
    hipLaunchKernelGGL(k_objects_l, dim3(std::max(1, n_cu / 4)), dim3(4 * WAVE), lds_l, u, args_dev, L);
    RT_HIP(hipGetLastError());
    if ((e = mark(2, 1, u)) || (e = mark(1, 0, s))) return e;
    hipLaunchKernelGGL(k_objects_m, dim3(n_cu * 4), dim3(2 * WAVE), lds_m, s, args_dev, L);
    RT_HIP(hipGetLastError());
    if ((e = mark(1, 1, s)) || (e = mark(0, 0, t))) return e;
    hipLaunchKernelGGL(k_objects_s1, dim3(n_cu * 32), dim3(WAVE), 0, t, args_dev, L);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_objects_s, dim3(n_cu * 24), dim3(WAVE), lds_s, t, args_dev, L);
    RT_HIP(hipGetLastError());
    if ((e = mark(0, 1, t))) return e;
    if (t != s) {
        RT_HIP(hipEventRecord(par->join, t));
        RT_HIP(hipStreamWaitEvent(s, par->join, 0));
        RT_HIP(hipEventRecord(par->join2, u));
        RT_HIP(hipStreamWaitEvent(s, par->join2, 0));
    }
    if (before_big) RT_HIP(hipEventRecord(before_big, s));
    BigPass mid{L.big, L.n_big, L.huge, L.n_huge, (char *)L.mid_scratch, L.mid_slice_bytes, MID_MAX_PX};
    hipLaunchKernelGGL(k_objects_big, dim3(L.mid_slices), dim3(WAVE), 0, s, args_dev, mid);
    RT_HIP(hipGetLastError());
    BigPass huge{L.huge, L.n_huge, nullptr, nullptr, (char *)L.big_scratch, L.big_slice_bytes, 0};
    hipLaunchKernelGGL(k_objects_big, dim3(L.big_slices), dim3(WAVE), 0, s, args_dev, huge);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rtseg
