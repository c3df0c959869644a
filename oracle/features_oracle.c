/*
 * features_oracle.c -- plain CPU oracle of the feature-computation stage
 * (Sec. 5.1 "Example Application": a set of shape and texture features per
 * segmented nucleus, computed from per-nucleus histograms and co-occurrence
 * matrices; Fig. 1: 60-100 shape and texture features per object).
 * TEST INFRASTRUCTURE ONLY (see rt_oracle.h).  Build with -ffp-contract=off.
 *
 * One raster pass over the tile accumulates every per-nucleus count
 * (histograms, co-occurrence matrix, coordinate sums, perimeter edges,
 * gradient sums), then each feature is evaluated from its textbook
 * definition, nucleus by nucleus.  Definitions and readings: rt_oracle.h.
 */
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "rt_oracle.h"

typedef struct {
    int32_t label;
    int64_t area, perim;
    int32_t x0, y0, x1, y1;
    int32_t xr, yr;                     /* the first pixel (row-major) */
    int64_t sx, sy, sxx, syy, sxy;      /* sums of coordinates relative to the first pixel */
    int64_t hist[256];                  /* Hq histogram */
    int64_t ghist[OR_GRAD_BINS];        /* Sobel magnitude histogram */
    int64_t gsum, gsum2, gmax;
    int64_t glcm[OR_GLCM_LEVELS][OR_GLCM_LEVELS];
} nuc_acc;

static int hq_at(const uint8_t *hq, int w, int h, int x, int y) {
    /* replicate the nearest edge pixel outside the tile */
    if (x < 0) x = 0;
    if (x >= w) x = w - 1;
    if (y < 0) y = 0;
    if (y >= h) y = h - 1;
    return hq[(int64_t)y * w + x];
}

static int64_t isqrt64(int64_t n) {
    if (n <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)n);
    while (r * r > n) --r;
    while ((r + 1) * (r + 1) <= n) ++r;
    return r;
}

int64_t or_sobel_mag(const uint8_t *hq, int w, int h, int x, int y) {
    /* gx = sum of the right column - sum of the left column with weights 1,2,1;
       gy = bottom row - top row with weights 1,2,1 */
    int gx = 0, gy = 0;
    for (int d = -1; d <= 1; ++d) {
        const int wt = d == 0 ? 2 : 1;
        gx += wt * (hq_at(hq, w, h, x + 1, y + d) - hq_at(hq, w, h, x - 1, y + d));
        gy += wt * (hq_at(hq, w, h, x + d, y + 1) - hq_at(hq, w, h, x + d, y - 1));
    }
    return isqrt64((int64_t)gx * gx + (int64_t)gy * gy);
}

static double plog2p(double p) { return p > 0.0 ? p * log2(p) : 0.0; }

/* value at 0-based rank r of the sorted pixel values */
static int rank_value(const int64_t *hist, int64_t r) {
    int64_t c = 0;
    for (int v = 0; v < 256; ++v) {
        c += hist[v];
        if (c > r) return v;
    }
    return 255;
}

static void features_of(const nuc_acc *n, double *f) {
    const double A = (double)n->area;
    const double PI = 3.14159265358979323846;
    /* ---- shape */
    f[OF_AREA] = A;
    f[OF_PERIMETER] = (double)n->perim;
    f[OF_CENTROID_X] = n->xr + (double)n->sx / A;
    f[OF_CENTROID_Y] = n->yr + (double)n->sy / A;
    const double bw = n->x1 - n->x0 + 1, bh = n->y1 - n->y0 + 1;
    f[OF_BBOX_W] = bw;
    f[OF_BBOX_H] = bh;
    f[OF_EXTENT] = A / (bw * bh);
    f[OF_EQUIV_DIAMETER] = sqrt(4.0 * A / PI);
    f[OF_CIRCULARITY] = 4.0 * PI * A / ((double)n->perim * (double)n->perim);
    /* second central moments of the pixel set, each pixel a unit square
       (variance 1/12 along each axis added) */
    /* A^2 mu = A sum x^2 - (sum x)^2, exact in 128-bit integers */
    const __int128 c20 = (__int128)n->area * n->sxx - (__int128)n->sx * n->sx;
    const __int128 c02 = (__int128)n->area * n->syy - (__int128)n->sy * n->sy;
    const __int128 c11 = (__int128)n->area * n->sxy - (__int128)n->sx * n->sy;
    const double AA = (double)(n->area * n->area);
    const double m20 = (double)c20 / AA + 1.0 / 12.0;
    const double m02 = (double)c02 / AA + 1.0 / 12.0;
    const double m11 = (double)c11 / AA;
    const double tr = m20 + m02;
    const double disc = sqrt((m20 - m02) * (m20 - m02) + 4.0 * m11 * m11);
    const double l1 = (tr + disc) / 2.0, l2 = (tr - disc) / 2.0;
    f[OF_MAJOR_AXIS] = 4.0 * sqrt(l1);
    f[OF_MINOR_AXIS] = 4.0 * sqrt(l2 > 0.0 ? l2 : 0.0);
    f[OF_ECCENTRICITY] = l1 > 0.0 ? sqrt(1.0 - (l2 > 0.0 ? l2 : 0.0) / l1) : 0.0;
    f[OF_ORIENTATION] = 0.5 * atan2(2.0 * m11, m20 - m02);
    /* ---- intensity of Hq over the nucleus */
    int64_t s1 = 0;
    int vmin = 255, vmax = 0;
    for (int v = 0; v < 256; ++v)
        if (n->hist[v]) {
            s1 += n->hist[v] * v;
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
        }
    const double mean = (double)s1 / A;
    double m2 = 0.0, m3 = 0.0, m4 = 0.0, ent = 0.0, en = 0.0;
    for (int v = 0; v < 256; ++v) {
        if (!n->hist[v]) continue;
        const double p = (double)n->hist[v] / A, d = v - mean;
        m2 += p * d * d;
        m3 += p * d * d * d;
        m4 += p * d * d * d * d;
        ent -= plog2p(p);
        en += p * p;
    }
    const double sd = sqrt(m2);
    f[OF_INT_MEAN] = mean;
    f[OF_INT_STD] = sd;
    f[OF_INT_MIN] = vmin;
    f[OF_INT_MAX] = vmax;
    f[OF_INT_MEDIAN] = rank_value(n->hist, (n->area - 1) / 2);
    f[OF_INT_P25] = rank_value(n->hist, (n->area - 1) / 4);
    f[OF_INT_P75] = rank_value(n->hist, 3 * (n->area - 1) / 4);
    f[OF_INT_SKEWNESS] = m2 > 0.0 ? m3 / (m2 * sd) : 0.0;
    f[OF_INT_KURTOSIS] = m2 > 0.0 ? m4 / (m2 * m2) : 0.0;
    f[OF_INT_ENTROPY] = ent;
    f[OF_INT_ENERGY] = en;
    f[OF_INT_RANGE] = vmax - vmin;
    /* ---- gradient magnitude over the nucleus */
    f[OF_GRAD_MEAN] = (double)n->gsum / A;
    f[OF_GRAD_STD] = sqrt((double)((__int128)n->area * n->gsum2 - (__int128)n->gsum * n->gsum)) / A;
    f[OF_GRAD_MAX] = (double)n->gmax;
    double gent = 0.0, gen = 0.0;
    int64_t edge = 0;
    for (int b = 0; b < OR_GRAD_BINS; ++b) {
        const double p = (double)n->ghist[b] / A;
        gent -= plog2p(p);
        gen += p * p;
        if (b * OR_GRAD_BIN_WIDTH >= OR_EDGE_THRESHOLD) edge += n->ghist[b];
    }
    f[OF_GRAD_ENTROPY] = gent;
    f[OF_GRAD_ENERGY] = gen;
    f[OF_EDGE_FRACTION] = (double)edge / A;
    /* ---- Haralick texture of the pooled symmetric co-occurrence matrix */
    const int G = OR_GLCM_LEVELS;
    int64_t tot = 0;
    for (int i = 0; i < G; ++i)
        for (int j = 0; j < G; ++j) tot += n->glcm[i][j];
    for (int k = OF_GLCM_ASM; k <= OF_GLCM_CLUSTER_PROMINENCE; ++k) f[k] = 0.0;
    if (tot == 0) return;
    double p[OR_GLCM_LEVELS][OR_GLCM_LEVELS], px[OR_GLCM_LEVELS];
    double psum[2 * OR_GLCM_LEVELS - 1], pdif[OR_GLCM_LEVELS];
    memset(px, 0, sizeof px);
    memset(psum, 0, sizeof psum);
    memset(pdif, 0, sizeof pdif);
    for (int i = 0; i < G; ++i)
        for (int j = 0; j < G; ++j) {
            p[i][j] = (double)n->glcm[i][j] / (double)tot;
            px[i] += p[i][j];
            psum[i + j] += p[i][j];
            pdif[abs(i - j)] += p[i][j];
        }
    /* the matrix is symmetric, so the column marginal equals px */
    double mu = 0.0;
    for (int i = 0; i < G; ++i) mu += i * px[i];
    double var = 0.0;
    for (int i = 0; i < G; ++i) var += (i - mu) * (i - mu) * px[i];
    double asm_ = 0.0, con = 0.0, cor = 0.0, hom = 0.0, entr = 0.0, mp = 0.0, shade = 0.0, prom = 0.0, hxy1 = 0.0,
           hxy2 = 0.0;
    for (int i = 0; i < G; ++i)
        for (int j = 0; j < G; ++j) {
            const double q = p[i][j];
            asm_ += q * q;
            con += (double)((i - j) * (i - j)) * q;
            cor += (i - mu) * (j - mu) * q;
            hom += q / (1.0 + (double)((i - j) * (i - j)));
            entr -= plog2p(q);
            if (q > mp) mp = q;
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
    for (int k = 0; k < 2 * G - 1; ++k) {
        savg += k * psum[k];
        sent -= plog2p(psum[k]);
    }
    double svar = 0.0;
    for (int k = 0; k < 2 * G - 1; ++k) svar += (k - savg) * (k - savg) * psum[k];
    double dmean = 0.0, dent = 0.0;
    for (int k = 0; k < G; ++k) {
        dmean += k * pdif[k];
        dent -= plog2p(pdif[k]);
    }
    double dvar = 0.0;
    for (int k = 0; k < G; ++k) dvar += (k - dmean) * (k - dmean) * pdif[k];
    f[OF_GLCM_ASM] = asm_;
    f[OF_GLCM_CONTRAST] = con;
    f[OF_GLCM_CORRELATION] = var > 0.0 ? cor / var : 1.0;
    f[OF_GLCM_VARIANCE] = var;
    f[OF_GLCM_HOMOGENEITY] = hom;
    f[OF_GLCM_SUM_AVERAGE] = savg;
    f[OF_GLCM_SUM_VARIANCE] = svar;
    f[OF_GLCM_SUM_ENTROPY] = sent;
    f[OF_GLCM_ENTROPY] = entr;
    f[OF_GLCM_DIFF_VARIANCE] = dvar;
    f[OF_GLCM_DIFF_ENTROPY] = dent;
    f[OF_GLCM_IMC1] = hx > 0.0 ? (entr - hxy1) / hx : 0.0;
    const double e2 = hxy2 - entr;
    f[OF_GLCM_IMC2] = sqrt(1.0 - exp(-2.0 * (e2 > 0.0 ? e2 : 0.0)));
    f[OF_GLCM_MAX_PROB] = mp;
    f[OF_GLCM_CLUSTER_SHADE] = shade;
    f[OF_GLCM_CLUSTER_PROMINENCE] = prom;
}

int or_features(const int32_t *labels, const uint8_t *hq, int w, int h, int max_nuclei, int32_t *labels_out,
                double *feats_out, int64_t *counts_out) {
    const int64_t N = (int64_t)w * h;
    /* label value -> nucleus index (labels are 1 + the row-major index of the
       nucleus' first pixel, so a nucleus is met first at that pixel) */
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    int cap = 64, n = 0;
    nuc_acc *acc = (nuc_acc *)malloc(sizeof(nuc_acc) * cap);
    for (int64_t i = 0; i <= N; ++i) idx[i] = -1;
    static const int ODX[4] = {1, 1, 0, -1}, ODY[4] = {0, 1, 1, 1};   /* 0, 45, 90, 135 degrees */
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const int64_t p = (int64_t)y * w + x;
            const int32_t L = labels[p];
            if (L <= 0) continue;
            if (idx[L] < 0) {
                if (n == cap) {
                    cap *= 2;
                    acc = (nuc_acc *)realloc(acc, sizeof(nuc_acc) * cap);
                }
                memset(&acc[n], 0, sizeof(nuc_acc));
                acc[n].label = L;
                acc[n].x0 = acc[n].x1 = acc[n].xr = x;
                acc[n].y0 = acc[n].y1 = acc[n].yr = y;
                idx[L] = n++;
            }
            nuc_acc *a = &acc[idx[L]];
            a->area += 1;
            if (x < a->x0) a->x0 = x;
            if (x > a->x1) a->x1 = x;
            if (y > a->y1) a->y1 = y;
            const int64_t dx = x - a->xr, dy = y - a->yr;
            a->sx += dx;
            a->sy += dy;
            a->sxx += dx * dx;
            a->syy += dy * dy;
            a->sxy += dx * dy;
            /* perimeter: 4-neighbour sides facing another label or the outside */
            static const int PX4[4] = {1, -1, 0, 0}, PY4[4] = {0, 0, 1, -1};
            for (int k = 0; k < 4; ++k) {
                const int xx = x + PX4[k], yy = y + PY4[k];
                if (xx < 0 || xx >= w || yy < 0 || yy >= h || labels[(int64_t)yy * w + xx] != L) a->perim += 1;
            }
            const int v = hq[p];
            a->hist[v] += 1;
            const int64_t g = or_sobel_mag(hq, w, h, x, y);
            a->gsum += g;
            a->gsum2 += g * g;
            if (g > a->gmax) a->gmax = g;
            int gb = (int)(g / OR_GRAD_BIN_WIDTH);
            if (gb > OR_GRAD_BINS - 1) gb = OR_GRAD_BINS - 1;
            a->ghist[gb] += 1;
            /* co-occurrence: each unordered pair of same-nucleus pixels at one
               of the four offsets, counted both ways */
            for (int k = 0; k < 4; ++k) {
                const int xx = x + ODX[k], yy = y + ODY[k];
                if (xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
                const int64_t q = (int64_t)yy * w + xx;
                if (labels[q] != L) continue;
                const int a1 = v / (256 / OR_GLCM_LEVELS), a2 = hq[q] / (256 / OR_GLCM_LEVELS);
                a->glcm[a1][a2] += 1;
                a->glcm[a2][a1] += 1;
            }
        }
    /* nuclei in increasing label order (the order of first pixels) */
    const int nout = n < max_nuclei ? n : max_nuclei;
    for (int k = 0; k < nout; ++k) {
        labels_out[k] = acc[k].label;
        features_of(&acc[k], feats_out + (int64_t)k * OR_NFEAT);
        if (counts_out) {
            int64_t *c = counts_out + (int64_t)k * OR_NCOUNT;
            c[0] = acc[k].area;
            c[1] = acc[k].perim;
            c[2] = acc[k].x0;
            c[3] = acc[k].y0;
            c[4] = acc[k].x1;
            c[5] = acc[k].y1;
            for (int v = 0; v < 256; ++v) c[6 + v] = acc[k].hist[v];
            for (int i = 0; i < OR_GLCM_LEVELS; ++i)
                for (int j = 0; j < OR_GLCM_LEVELS; ++j) c[262 + i * OR_GLCM_LEVELS + j] = acc[k].glcm[i][j];
            for (int b = 0; b < OR_GRAD_BINS; ++b) c[518 + b] = acc[k].ghist[b];
            c[534] = acc[k].gsum;
            c[535] = acc[k].gsum2;
            c[536] = acc[k].gmax;
        }
    }
    free(idx);
    free(acc);
    return n;
}
