// Feature computation (Sec. 5.1): per-nucleus shape, intensity, gradient and
// Haralick texture features, in the paper's two steps -- one block per
// nucleus bounding box builds the nucleus' histograms, co-occurrence matrix
// and coordinate/gradient sums (fixed-size intermediates), then one thread
// per nucleus evaluates the features from them.
//
// Before the two steps, three light passes find the nuclei and their boxes
// without per-pixel atomics: a nucleus' label is 1 + the row-major index of
// its first pixel (its "root"), so
//   rows      one wave per row counts the root pixels of the row;
//   scan      one block turns the counts into row offsets (ranks in label
//             order) and the total;
//   register  one wave per row writes each root's rank into a label -> rank
//             map (only at root positions; the map is never cleared, a lookup
//             is checked against the registered label), the label list and
//             the box seed (the root's x, y);
//   boxes     one wave per 64-pixel row chunk finds the label runs of the
//             chunk (ballots) and widens the run's nucleus box with three
//             atomics per run.
#include "rt_internal.h"

namespace rtseg {

namespace {

constexpr int FW = 64;   // wave size

__device__ __forceinline__ int32_t lab_at(const FeatArgs &a, int x, int y) {
    return a.labels[(int64_t)y * a.lab_pitch + x];
}

// rank of the nucleus with label L, or -1 when L was not registered
__device__ __forceinline__ int lookup(const FeatArgs &a, int32_t L, int n_reg) {
    if (L <= 0 || (int64_t)L > (int64_t)a.w * a.h) return -1;
    const int k = a.map[L - 1];
    if (k < 0 || k >= n_reg) return -1;
    return a.labels_out[k] == L ? k : -1;
}

__global__ __launch_bounds__(256) void k_feat_rows(FeatArgs a) {
    const int lane = threadIdx.x & (FW - 1);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / FW;
    const int nwaves = gridDim.x * blockDim.x / FW;
    for (int y = wave; y < a.h; y += nwaves) {
        int cnt = 0;
        for (int x0 = 0; x0 < a.w; x0 += FW) {
            const int x = x0 + lane;
            const bool root = x < a.w && lab_at(a, x, y) == y * a.w + x + 1;
            cnt += __popcll(__ballot(root));
        }
        if (lane == 0) a.row_off[y] = cnt;
    }
}

// exclusive scan of row_off[0..h) in place; row_off[h] = total
__global__ __launch_bounds__(1024) void k_feat_scan(FeatArgs a) {
    __shared__ int part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int seg = (a.h + nt - 1) / nt;
    const int b = min(a.h, t * seg), e = min(a.h, b + seg);
    int s = 0;
    for (int y = b; y < e; ++y) s += a.row_off[y];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {   // inclusive Hillis-Steele scan
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int y = b; y < e; ++y) {
        const int c = a.row_off[y];
        a.row_off[y] = run;
        run += c;
    }
    if (t == nt - 1) {
        a.row_off[a.h] = part[t];
        if (a.n_out) *a.n_out = part[t];
    }
}

__global__ __launch_bounds__(256) void k_feat_register(FeatArgs a) {
    const int lane = threadIdx.x & (FW - 1);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / FW;
    const int nwaves = gridDim.x * blockDim.x / FW;
    const uint64_t below = (1ull << lane) - 1;
    for (int y = wave; y < a.h; y += nwaves) {
        int base = a.row_off[y];
        if (base >= a.max_nuclei) continue;
        for (int x0 = 0; x0 < a.w; x0 += FW) {
            const int x = x0 + lane;
            const int32_t L = x < a.w ? lab_at(a, x, y) : 0;
            const bool root = x < a.w && L == y * a.w + x + 1;
            const uint64_t m = __ballot(root);
            const int r = base + __popcll(m & below);
            if (root && r < a.max_nuclei) {
                a.labels_out[r] = L;
                a.map[L - 1] = r;
                a.box[4 * r + 0] = x;
                a.box[4 * r + 1] = y;
                a.box[4 * r + 2] = x;
                a.box[4 * r + 3] = y;
            }
            base += __popcll(m);
        }
    }
}

__global__ __launch_bounds__(256) void k_feat_boxes(FeatArgs a) {
    const int lane = threadIdx.x & (FW - 1);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / FW;
    const int nwaves = gridDim.x * blockDim.x / FW;
    const int n_reg = min(a.row_off[a.h], a.max_nuclei);
    const int chunks = (a.w + FW - 1) / FW;
    const int64_t units = (int64_t)a.h * chunks;
    for (int64_t u = wave; u < units; u += nwaves) {
        const int y = (int)(u / chunks), x = (int)(u % chunks) * FW + lane;
        const int32_t L = x < a.w ? lab_at(a, x, y) : 0;
        const int32_t Ll = __shfl_up(L, 1), Lr = __shfl_down(L, 1);
        const bool start = L > 0 && (lane == 0 || Ll != L);
        const bool end = L > 0 && (lane == FW - 1 || x == a.w - 1 || Lr != L);
        const uint64_t ends = __ballot(end);
        if (start) {
            const int k = lookup(a, L, n_reg);
            if (k >= 0) {
                const uint64_t after = ends >> lane;   // bit 0 = this lane
                const int xe = x + (int)__builtin_ctzll(after);
                atomicMin(a.box + 4 * k + 0, x);
                atomicMax(a.box + 4 * k + 2, xe);
                atomicMax(a.box + 4 * k + 3, y);
            }
        }
    }
}

__device__ __forceinline__ int hq_clamped(const FeatArgs &a, int x, int y) {
    x = min(max(x, 0), a.w - 1);
    y = min(max(y, 0), a.h - 1);
    return a.hq[(int64_t)y * a.hq_pitch + x];
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ __forceinline__ int64_t wave_max64(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int64_t o = __shfl_xor(v, d);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int isqrt_i(int v) {
    int r = (int)sqrtf((float)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// step 1: one wave per nucleus box
__global__ __launch_bounds__(FW) void k_feat_accum(FeatArgs a) {
    __shared__ uint32_t hist[256], glcm[256], ghist[RT_FEAT_GRAD_BINS];
    const int lane = threadIdx.x;
    const int n_reg = min(a.row_off[a.h], a.max_nuclei);
    constexpr int QS = 256 / RT_FEAT_GLCM_LEVELS;   // Hq / QS = grey level
    for (int k = blockIdx.x; k < n_reg; k += gridDim.x) {
        for (int i = lane; i < 256; i += FW) {
            hist[i] = 0;
            glcm[i] = 0;
        }
        if (lane < RT_FEAT_GRAD_BINS) ghist[lane] = 0;
        __syncthreads();
        const int32_t L = a.labels_out[k];
        const int xr = (L - 1) % a.w, yr = (L - 1) / a.w;
        const int bx0 = a.box[4 * k + 0], by0 = a.box[4 * k + 1], bx1 = a.box[4 * k + 2], by1 = a.box[4 * k + 3];
        const int bw = bx1 - bx0 + 1;
        const int64_t npx = (int64_t)bw * (by1 - by0 + 1);
        int64_t area = 0, perim = 0, sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0, gs = 0, gs2 = 0, gmax = 0;
        for (int64_t i = lane; i < npx; i += FW) {
            const int x = bx0 + (int)(i % bw), y = by0 + (int)(i / bw);
            if (lab_at(a, x, y) != L) continue;
            // neighbour labels (0 outside the tile)
            const int32_t lr = x + 1 < a.w ? lab_at(a, x + 1, y) : 0;
            const int32_t ll = x > 0 ? lab_at(a, x - 1, y) : 0;
            const int32_t ld = y + 1 < a.h ? lab_at(a, x, y + 1) : 0;
            const int32_t lu = y > 0 ? lab_at(a, x, y - 1) : 0;
            const int32_t ldr = (x + 1 < a.w && y + 1 < a.h) ? lab_at(a, x + 1, y + 1) : 0;
            const int32_t ldl = (x > 0 && y + 1 < a.h) ? lab_at(a, x - 1, y + 1) : 0;
            // 3 x 3 Hq neighbourhood, replicated at the tile edge
            int q[3][3];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) q[dy + 1][dx + 1] = hq_clamped(a, x + dx, y + dy);
            area += 1;
            perim += (lr != L) + (ll != L) + (ld != L) + (lu != L);
            const int64_t dx = x - xr, dy = y - yr;
            sx += dx;
            sy += dy;
            sxx += dx * dx;
            syy += dy * dy;
            sxy += dx * dy;
            const int v = q[1][1];
            atomicAdd(hist + v, 1u);
            const int gx = (q[0][2] - q[0][0]) + 2 * (q[1][2] - q[1][0]) + (q[2][2] - q[2][0]);
            const int gy = (q[2][0] - q[0][0]) + 2 * (q[2][1] - q[0][1]) + (q[2][2] - q[0][2]);
            const int g = isqrt_i(gx * gx + gy * gy);
            gs += g;
            gs2 += (int64_t)g * g;
            gmax = g > gmax ? g : gmax;
            atomicAdd(ghist + min(g / RT_FEAT_GRAD_BIN_WIDTH, RT_FEAT_GRAD_BINS - 1), 1u);
            // co-occurrence at 0, 45, 90, 135 degrees (forward neighbours), both orders
            const int a1 = v / QS;
            if (lr == L) {
                const int a2 = q[1][2] / QS;
                atomicAdd(glcm + a1 * RT_FEAT_GLCM_LEVELS + a2, 1u);
                atomicAdd(glcm + a2 * RT_FEAT_GLCM_LEVELS + a1, 1u);
            }
            if (ldr == L) {
                const int a2 = q[2][2] / QS;
                atomicAdd(glcm + a1 * RT_FEAT_GLCM_LEVELS + a2, 1u);
                atomicAdd(glcm + a2 * RT_FEAT_GLCM_LEVELS + a1, 1u);
            }
            if (ld == L) {
                const int a2 = q[2][1] / QS;
                atomicAdd(glcm + a1 * RT_FEAT_GLCM_LEVELS + a2, 1u);
                atomicAdd(glcm + a2 * RT_FEAT_GLCM_LEVELS + a1, 1u);
            }
            if (ldl == L) {
                const int a2 = q[2][0] / QS;
                atomicAdd(glcm + a1 * RT_FEAT_GLCM_LEVELS + a2, 1u);
                atomicAdd(glcm + a2 * RT_FEAT_GLCM_LEVELS + a1, 1u);
            }
        }
        area = wave_sum64(area);
        perim = wave_sum64(perim);
        sx = wave_sum64(sx);
        sy = wave_sum64(sy);
        sxx = wave_sum64(sxx);
        syy = wave_sum64(syy);
        sxy = wave_sum64(sxy);
        gs = wave_sum64(gs);
        gs2 = wave_sum64(gs2);
        gmax = wave_max64(gmax);
        __syncthreads();
        NucAcc *o = a.acc + k;
        if (lane == 0) {
            o->area = area;
            o->perim = perim;
            o->sx = sx;
            o->sy = sy;
            o->sxx = sxx;
            o->syy = syy;
            o->sxy = sxy;
            o->gsum = gs;
            o->gsum2 = gs2;
            o->gmax = gmax;
        }
        for (int i = lane; i < 256; i += FW) {
            o->hist[i] = hist[i];
            o->glcm[i] = glcm[i];
        }
        if (lane < RT_FEAT_GRAD_BINS) o->ghist[lane] = ghist[lane];
        __syncthreads();
    }
}

__device__ __forceinline__ double plog2p(double p) { return p > 0.0 ? p * log2(p) : 0.0; }

__device__ int rank_value(const uint32_t *hist, int64_t r) {
    int64_t c = 0;
    for (int v = 0; v < 256; ++v) {
        c += hist[v];
        if (c > r) return v;
    }
    return 255;
}

// step 2: one thread per nucleus
__global__ __launch_bounds__(64) void k_feat_finish(FeatArgs a) {
    const int n_reg = min(a.row_off[a.h], a.max_nuclei);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_reg) return;
    const NucAcc *n = a.acc + k;
    double *f = a.feats + (int64_t)k * RT_NFEAT;
    const int32_t L = a.labels_out[k];
    const int xr = (L - 1) % a.w, yr = (L - 1) / a.w;
    const int bx0 = a.box[4 * k + 0], by0 = a.box[4 * k + 1], bx1 = a.box[4 * k + 2], by1 = a.box[4 * k + 3];
    const int64_t area = n->area;
    const double A = (double)area;
    const double PI = 3.14159265358979323846;
    // ---- shape
    f[0] = A;
    f[1] = (double)n->perim;
    f[2] = xr + (double)n->sx / A;
    f[3] = yr + (double)n->sy / A;
    const double bw = bx1 - bx0 + 1, bh = by1 - by0 + 1;
    f[4] = bw;
    f[5] = bh;
    f[6] = A / (bw * bh);
    f[7] = sqrt(4.0 * A / PI);
    f[8] = 4.0 * PI * A / ((double)n->perim * (double)n->perim);
    const __int128 c20 = (__int128)area * n->sxx - (__int128)n->sx * n->sx;
    const __int128 c02 = (__int128)area * n->syy - (__int128)n->sy * n->sy;
    const __int128 c11 = (__int128)area * n->sxy - (__int128)n->sx * n->sy;
    const double AA = (double)(area * area);
    const double m20 = (double)c20 / AA + 1.0 / 12.0;
    const double m02 = (double)c02 / AA + 1.0 / 12.0;
    const double m11 = (double)c11 / AA;
    const double tr = m20 + m02;
    const double disc = sqrt((m20 - m02) * (m20 - m02) + 4.0 * m11 * m11);
    const double l1 = (tr + disc) / 2.0, l2 = (tr - disc) / 2.0;
    f[9] = 4.0 * sqrt(l1);
    f[10] = 4.0 * sqrt(l2 > 0.0 ? l2 : 0.0);
    f[11] = l1 > 0.0 ? sqrt(1.0 - (l2 > 0.0 ? l2 : 0.0) / l1) : 0.0;
    f[12] = 0.5 * atan2(2.0 * m11, m20 - m02);
    // ---- intensity
    int64_t s1 = 0;
    int vmin = 255, vmax = 0;
    for (int v = 0; v < 256; ++v)
        if (n->hist[v]) {
            s1 += (int64_t)n->hist[v] * v;
            vmin = v < vmin ? v : vmin;
            vmax = v > vmax ? v : vmax;
        }
    const double mean = (double)s1 / A;
    double m2 = 0.0, m3 = 0.0, m4 = 0.0, ent = 0.0, en = 0.0;
    for (int v = 0; v < 256; ++v) {
        const uint32_t c = n->hist[v];
        if (!c) continue;
        const double p = (double)c / A, d = v - mean;
        m2 += p * d * d;
        m3 += p * d * d * d;
        m4 += p * d * d * d * d;
        ent -= plog2p(p);
        en += p * p;
    }
    const double sd = sqrt(m2);
    f[13] = mean;
    f[14] = sd;
    f[15] = vmin;
    f[16] = vmax;
    f[17] = rank_value(n->hist, (area - 1) / 2);
    f[18] = rank_value(n->hist, (area - 1) / 4);
    f[19] = rank_value(n->hist, 3 * (area - 1) / 4);
    f[20] = m2 > 0.0 ? m3 / (m2 * sd) : 0.0;
    f[21] = m2 > 0.0 ? m4 / (m2 * m2) : 0.0;
    f[22] = ent;
    f[23] = en;
    f[24] = vmax - vmin;
    // ---- gradient
    f[25] = (double)n->gsum / A;
    f[26] = sqrt((double)((__int128)area * n->gsum2 - (__int128)n->gsum * n->gsum)) / A;
    f[27] = (double)n->gmax;
    double gent = 0.0, gen = 0.0;
    int64_t edge = 0;
    for (int b = 0; b < RT_FEAT_GRAD_BINS; ++b) {
        const double p = (double)n->ghist[b] / A;
        gent -= plog2p(p);
        gen += p * p;
        if (b * RT_FEAT_GRAD_BIN_WIDTH >= RT_FEAT_EDGE_THRESHOLD) edge += n->ghist[b];
    }
    f[28] = gent;
    f[29] = gen;
    f[30] = (double)edge / A;
    // ---- Haralick texture of the pooled co-occurrence matrix
    constexpr int G = RT_FEAT_GLCM_LEVELS;
    int64_t tot = 0;
    for (int i = 0; i < G * G; ++i) tot += n->glcm[i];
    for (int i = 31; i < RT_NFEAT; ++i) f[i] = 0.0;
    if (tot == 0) return;
    const double T = (double)tot;
    double px[G], psum[2 * G - 1], pdif[G];
    for (int i = 0; i < G; ++i) px[i] = pdif[i] = 0.0;
    for (int i = 0; i < 2 * G - 1; ++i) psum[i] = 0.0;
    for (int i = 0; i < G; ++i)
        for (int j = 0; j < G; ++j) {
            const double p = (double)n->glcm[i * G + j] / T;
            px[i] += p;
            psum[i + j] += p;
            pdif[i > j ? i - j : j - i] += p;
        }
    double mu = 0.0;
    for (int i = 0; i < G; ++i) mu += i * px[i];
    double var = 0.0;
    for (int i = 0; i < G; ++i) var += (i - mu) * (i - mu) * px[i];
    double asm_ = 0.0, con = 0.0, cor = 0.0, hom = 0.0, entr = 0.0, mp = 0.0, shade = 0.0, prom = 0.0, hxy1 = 0.0,
           hxy2 = 0.0;
    for (int i = 0; i < G; ++i)
        for (int j = 0; j < G; ++j) {
            const double q = (double)n->glcm[i * G + j] / T;
            asm_ += q * q;
            con += (double)((i - j) * (i - j)) * q;
            cor += (i - mu) * (j - mu) * q;
            hom += q / (1.0 + (double)((i - j) * (i - j)));
            entr -= plog2p(q);
            mp = q > mp ? q : mp;
            const double s = i + j - 2.0 * mu;
            shade += s * s * s * q;
            prom += s * s * s * s * q;
            const double pp = px[i] * px[j];
            if (pp > 0.0) {
                hxy1 -= q * log2(pp);
                hxy2 -= pp * log2(pp);
            }
        }
    double hx = 0.0;
    for (int i = 0; i < G; ++i) hx -= plog2p(px[i]);
    double savg = 0.0, sent = 0.0;
    for (int i = 0; i < 2 * G - 1; ++i) {
        savg += i * psum[i];
        sent -= plog2p(psum[i]);
    }
    double svar = 0.0;
    for (int i = 0; i < 2 * G - 1; ++i) svar += (i - savg) * (i - savg) * psum[i];
    double dmean = 0.0, dent = 0.0;
    for (int i = 0; i < G; ++i) {
        dmean += i * pdif[i];
        dent -= plog2p(pdif[i]);
    }
    double dvar = 0.0;
    for (int i = 0; i < G; ++i) dvar += (i - dmean) * (i - dmean) * pdif[i];
    f[31] = asm_;
    f[32] = con;
    f[33] = var > 0.0 ? cor / var : 1.0;
    f[34] = var;
    f[35] = hom;
    f[36] = savg;
    f[37] = svar;
    f[38] = sent;
    f[39] = entr;
    f[40] = dvar;
    f[41] = dent;
    f[42] = hx > 0.0 ? (entr - hxy1) / hx : 0.0;
    const double e2 = hxy2 - entr;
    f[43] = sqrt(1.0 - exp(-2.0 * (e2 > 0.0 ? e2 : 0.0)));
    f[44] = mp;
    f[45] = shade;
    f[46] = prom;
}

// counts in the layout of the public header (int64 per entry)
__global__ __launch_bounds__(256) void k_feat_counts(FeatArgs a) {
    const int n_reg = min(a.row_off[a.h], a.max_nuclei);
    const int64_t total = (int64_t)n_reg * RT_FEAT_NCOUNT;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(i / RT_FEAT_NCOUNT), c = (int)(i % RT_FEAT_NCOUNT);
        const NucAcc *n = a.acc + k;
        int64_t v;
        if (c == 0)
            v = n->area;
        else if (c == 1)
            v = n->perim;
        else if (c < 6)
            v = a.box[4 * k + (c - 2)];
        else if (c < 262)
            v = n->hist[c - 6];
        else if (c < 518)
            v = n->glcm[c - 262];
        else if (c < 534)
            v = n->ghist[c - 518];
        else if (c == 534)
            v = n->gsum;
        else if (c == 535)
            v = n->gsum2;
        else
            v = n->gmax;
        a.counts[i] = v;
    }
}

}  // namespace

int launch_features(const FeatArgs &a, int n_cu, hipStream_t s) {
    const int row_blocks = std::max(1, std::min((a.h + 3) / 4, n_cu * 8));
    hipLaunchKernelGGL(k_feat_rows, dim3(row_blocks), dim3(256), 0, s, a);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_scan, dim3(1), dim3(1024), 0, s, a);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_register, dim3(row_blocks), dim3(256), 0, s, a);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_boxes, dim3(n_cu * 8), dim3(256), 0, s, a);
    RT_HIP(hipGetLastError());
    if (a.max_nuclei <= 0) return RT_OK;
    hipLaunchKernelGGL(k_feat_accum, dim3(std::min(a.max_nuclei, n_cu * 32)), dim3(FW), 0, s, a);
    RT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_finish, dim3((a.max_nuclei + 63) / 64), dim3(64), 0, s, a);
    RT_HIP(hipGetLastError());
    if (a.counts) {
        hipLaunchKernelGGL(k_feat_counts, dim3(n_cu * 4), dim3(256), 0, s, a);
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}

}  // namespace rtseg
