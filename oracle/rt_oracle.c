/*
 * rt_oracle.c -- plain CPU oracle for per-tile nucleus segmentation.
 * TEST INFRASTRUCTURE ONLY (see rt_oracle.h).  Build with -ffp-contract=off.
 *
 * Each function computes the definition stated in rt_oracle.h with a plain
 * sequential algorithm: breadth-first search, a binary heap for widest paths,
 * the separable exact distance transform.  No blocking, fusion or reordering.
 */
#include "rt_oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int DX8[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
static const int DY8[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int DX4[4] = {0, -1, 1, 0};
static const int DY4[4] = {-1, 0, 0, 1};

/* ------------------------------------------------------------------------ */
/* Colour deconvolution                                                     */
/* ------------------------------------------------------------------------ */

/* Column 0 of inv(M), M = [h; e; r] with normalised rows. */
static int stain_inverse_col0(const double rows[9], double m[3]) {
    double M[3][3];
    for (int i = 0; i < 3; ++i) {
        double n = sqrt(rows[3 * i] * rows[3 * i] + rows[3 * i + 1] * rows[3 * i + 1] +
                        rows[3 * i + 2] * rows[3 * i + 2]);
        for (int k = 0; k < 3; ++k) M[i][k] = (n > 0.0) ? rows[3 * i + k] / n : 0.0;
    }
    double n2 = M[2][0] * M[2][0] + M[2][1] * M[2][1] + M[2][2] * M[2][2];
    if (n2 == 0.0) {
        /* third stain = normalize(h x e) */
        double c0 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
        double c1 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
        double c2 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        double n = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        if (n == 0.0) return -1;
        M[2][0] = c0 / n;
        M[2][1] = c1 / n;
        M[2][2] = c2 / n;
    }
    /* inv(M) = adj(M) / det(M); column 0 of adj(M) is row 0 of the cofactor matrix. */
    double C00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    double C01 = -(M[1][0] * M[2][2] - M[1][2] * M[2][0]);
    double C02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    double det = M[0][0] * C00 + M[0][1] * C01 + M[0][2] * C02;
    if (det == 0.0) return -1;
    m[0] = C00 / det;
    m[1] = C01 / det;
    m[2] = C02 / det;
    return 0;
}

int or_deconv_od(const double stain_rows[9], const double od[3], double *cH) {
    double m[3];
    if (stain_inverse_col0(stain_rows, m)) return -1;
    double a = od[0] * m[0];
    double b = od[1] * m[1];
    double c = od[2] * m[2];
    *cH = (a + b) + c;
    return 0;
}

int or_deconv(const uint8_t *rgb, int w, int h, const double stain_rows[9], double scale,
              double *cH_out, uint8_t *hq_out) {
    double m[3];
    if (stain_inverse_col0(stain_rows, m)) return -1;
    double T[3][256];
    for (int k = 0; k < 3; ++k)
        for (int v = 0; v < 256; ++v) {
            double od = -log((double)(v + 1) / 256.0);
            T[k][v] = m[k] * od;
        }
    long n = (long)w * h;
    for (long i = 0; i < n; ++i) {
        double c = (T[0][rgb[3 * i]] + T[1][rgb[3 * i + 1]]) + T[2][rgb[3 * i + 2]];
        if (cH_out) cH_out[i] = c;
        double q = floor(c * scale + 0.5);
        if (q < 0.0) q = 0.0;
        if (q > 255.0) q = 255.0;
        hq_out[i] = (uint8_t)q;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Binary max-heap of (value, pixel) for widest paths                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t *a;
    long n, cap;
} heap_t;

static uint64_t hkey(int32_t v, int32_t idx) {
    return ((uint64_t)((uint32_t)v ^ 0x80000000u) << 32) | (uint32_t)idx;
}

static void hpush(heap_t *hp, uint64_t k) {
    if (hp->n == hp->cap) {
        hp->cap = hp->cap ? 2 * hp->cap : 1024;
        hp->a = (uint64_t *)realloc(hp->a, (size_t)hp->cap * sizeof(uint64_t));
    }
    long i = hp->n++;
    while (i > 0) {
        long p = (i - 1) / 2;
        if (hp->a[p] >= k) break;
        hp->a[i] = hp->a[p];
        i = p;
    }
    hp->a[i] = k;
}

static uint64_t hpop(heap_t *hp) {
    uint64_t top = hp->a[0];
    uint64_t last = hp->a[--hp->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1;
        if (l >= hp->n) break;
        long c = l;
        if (l + 1 < hp->n && hp->a[l + 1] > hp->a[l]) c = l + 1;
        if (hp->a[c] <= last) break;
        hp->a[i] = hp->a[c];
        i = c;
    }
    if (hp->n > 0) hp->a[i] = last;
    return top;
}

void or_recon(const int32_t *marker, const int32_t *mask, const uint8_t *domain, int w, int h,
              int conn, int32_t *out) {
    long n = (long)w * h;
    const int *dx = conn == 4 ? DX4 : DX8;
    const int *dy = conn == 4 ? DY4 : DY8;
    int nn = conn == 4 ? 4 : 8;
    uint8_t *done = (uint8_t *)calloc((size_t)n, 1);
    heap_t hp = {0, 0, 0};
    for (long p = 0; p < n; ++p) {
        out[p] = marker[p] < mask[p] ? marker[p] : mask[p];
        if (!domain || domain[p]) hpush(&hp, hkey(out[p], (int32_t)p));
    }
    while (hp.n > 0) {
        uint64_t k = hpop(&hp);
        int32_t p = (int32_t)(k & 0xffffffffu);
        int32_t v = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
        if (done[p] || v != out[p]) continue;
        done[p] = 1;
        int x = p % w, y = p / w;
        for (int d = 0; d < nn; ++d) {
            int qx = x + dx[d], qy = y + dy[d];
            if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
            long q = (long)qy * w + qx;
            if (done[q] || (domain && !domain[q])) continue;
            int32_t c = v < mask[q] ? v : mask[q];
            if (c > out[q]) {
                out[q] = c;
                hpush(&hp, hkey(c, (int32_t)q));
            }
        }
    }
    free(hp.a);
    free(done);
}

/* ------------------------------------------------------------------------ */
/* Hole filling and connected components (breadth-first search)             */
/* ------------------------------------------------------------------------ */

void or_fill_holes(const uint8_t *in, int w, int h, int bg_conn, uint8_t *out) {
    long n = (long)w * h;
    const int *dx = bg_conn == 8 ? DX8 : DX4;
    const int *dy = bg_conn == 8 ? DY8 : DY4;
    int nn = bg_conn == 8 ? 8 : 4;
    uint8_t *reach = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    long qh = 0, qt = 0;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            if (x != 0 && y != 0 && x != w - 1 && y != h - 1) continue;
            long p = (long)y * w + x;
            if (!in[p] && !reach[p]) {
                reach[p] = 1;
                queue[qt++] = (int32_t)p;
            }
        }
    while (qh < qt) {
        int32_t p = queue[qh++];
        int x = p % w, y = p / w;
        for (int d = 0; d < nn; ++d) {
            int qx = x + dx[d], qy = y + dy[d];
            if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
            long q = (long)qy * w + qx;
            if (!in[q] && !reach[q]) {
                reach[q] = 1;
                queue[qt++] = (int32_t)q;
            }
        }
    }
    for (long p = 0; p < n; ++p) out[p] = (in[p] || !reach[p]) ? 1 : 0;
    free(queue);
    free(reach);
}

int or_ccl(const uint8_t *mask, int w, int h, int conn, int32_t *labels) {
    long n = (long)w * h;
    const int *dx = conn == 4 ? DX4 : DX8;
    const int *dy = conn == 4 ? DY4 : DY8;
    int nn = conn == 4 ? 4 : 8;
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    memset(labels, 0, (size_t)n * sizeof(int32_t));
    int count = 0;
    for (long s = 0; s < n; ++s) {
        if (!mask[s] || labels[s]) continue;
        /* s is the first pixel of its component in row-major order, hence its
           smallest index. */
        int32_t lab = (int32_t)(s + 1);
        long qh = 0, qt = 0;
        labels[s] = lab;
        queue[qt++] = (int32_t)s;
        while (qh < qt) {
            int32_t p = queue[qh++];
            int x = p % w, y = p / w;
            for (int d = 0; d < nn; ++d) {
                int qx = x + dx[d], qy = y + dy[d];
                if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
                long q = (long)qy * w + qx;
                if (mask[q] && !labels[q]) {
                    labels[q] = lab;
                    queue[qt++] = (int32_t)q;
                }
            }
        }
        ++count;
    }
    free(queue);
    return count;
}

int or_area_filter(const int32_t *labels_in, int w, int h, int min_area, int max_area,
                   int32_t *labels_out, uint8_t *mask_out) {
    long n = (long)w * h;
    int32_t *area = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    for (long p = 0; p < n; ++p)
        if (labels_in[p] > 0) area[labels_in[p]]++;
    int kept = 0;
    for (long l = 1; l <= n; ++l)
        if (area[l] > 0 && area[l] >= min_area && area[l] <= max_area) ++kept;
    for (long p = 0; p < n; ++p) {
        int32_t l = labels_in[p];
        int32_t o = (l > 0 && area[l] >= min_area && area[l] <= max_area) ? l : 0;
        labels_out[p] = o;
        if (mask_out) mask_out[p] = o ? 1 : 0;
    }
    free(area);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Exact Euclidean distance transform                                       */
/* ------------------------------------------------------------------------ */

void or_edt_sq(const uint8_t *fg, int w, int h, int64_t *d2) {
    long n = (long)w * h;
    const int64_t INF = (int64_t)w + h + 1; /* larger than any in-tile distance */
    int64_t *g = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int any_zero = 0;
    /* column pass: distance to the nearest 0-pixel in the same column */
    for (int x = 0; x < w; ++x) {
        int64_t run = INF;
        for (int y = 0; y < h; ++y) {
            long p = (long)y * w + x;
            if (!fg[p]) {
                run = 0;
                any_zero = 1;
            } else if (run < INF)
                run++;
            g[p] = run;
        }
        run = INF;
        for (int y = h - 1; y >= 0; --y) {
            long p = (long)y * w + x;
            if (!fg[p])
                run = 0;
            else if (run < INF)
                run++;
            if (run < g[p]) g[p] = run;
        }
    }
    if (!any_zero) {
        for (long p = 0; p < n; ++p) d2[p] = -1;
        free(g);
        return;
    }
    /* row pass: lower envelope of parabolas f_u(x) = (x-u)^2 + g(u)^2 over the
       columns u with a finite column distance */
    int *v = (int *)malloc((size_t)w * sizeof(int));
    double *z = (double *)malloc((size_t)(w + 1) * sizeof(double));
    for (int y = 0; y < h; ++y) {
        const int64_t *gr = g + (long)y * w;
        int k = -1;
        for (int u = 0; u < w; ++u) {
            if (gr[u] >= INF) continue;
            double fu = (double)(gr[u] * gr[u] + (int64_t)u * u);
            if (k < 0) {
                k = 0;
                v[0] = u;
                z[0] = -HUGE_VAL;
                z[1] = HUGE_VAL;
                continue;
            }
            for (;;) {
                int vk = v[k];
                double fv = (double)(gr[vk] * gr[vk] + (int64_t)vk * vk);
                double s = (fu - fv) / (2.0 * (u - vk));
                if (s <= z[k] && k > 0) {
                    --k;
                    continue;
                }
                if (s <= z[k]) { /* k == 0: u dominates everywhere */
                    v[0] = u;
                    z[0] = -HUGE_VAL;
                    z[1] = HUGE_VAL;
                    break;
                }
                ++k;
                v[k] = u;
                z[k] = s;
                z[k + 1] = HUGE_VAL;
                break;
            }
        }
        int j = 0;
        for (int x = 0; x < w; ++x) {
            while (z[j + 1] < (double)x) ++j;
            long p = (long)y * w + x;
            if (!fg[p]) {
                d2[p] = 0;
                continue;
            }
            int64_t dxv = (int64_t)x - v[j];
            d2[p] = dxv * dxv + gr[v[j]] * gr[v[j]];
        }
    }
    free(z);
    free(v);
    free(g);
}

int64_t or_isqrt(int64_t n) {
    if (n <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)n);
    while (r * r > n) --r;
    while ((r + 1) * (r + 1) <= n) ++r;
    return r;
}

void or_dq(const uint8_t *fg, int w, int h, int32_t *dq) {
    long n = (long)w * h;
    int64_t *d2 = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    or_edt_sq(fg, w, h, d2);
    for (long p = 0; p < n; ++p) {
        if (!fg[p])
            dq[p] = 0;
        else if (d2[p] < 0)
            dq[p] = OR_DQ_MAX;
        else
            dq[p] = (int32_t)or_isqrt(4 * d2[p]);
    }
    free(d2);
}

/* ------------------------------------------------------------------------ */
/* Watershed                                                                */
/* ------------------------------------------------------------------------ */

static int cmp_desc_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x < y) - (x > y);
}

void or_watershed(const uint8_t *fg, const uint8_t *seeds, int h_seed, int w, int h,
                  int32_t *labels_out, uint8_t *mask_out,
                  int32_t *dq_out, int32_t *seed_lab_out, int32_t *lambda_out, int32_t *flood_out) {
    long n = (long)w * h;
    size_t nb = (size_t)(n > 0 ? n : 1);
    uint8_t *A = (uint8_t *)calloc(nb, 1);
    for (long p = 0; p < n; ++p) A[p] = fg[p] ? 1 : 0;
    int32_t *dq = (int32_t *)malloc(nb * sizeof(int32_t));
    or_dq(A, w, h, dq);

    /* seeds */
    uint8_t *rm = (uint8_t *)calloc(nb, 1);
    if (!seeds) {
        int32_t *mk = (int32_t *)malloc(nb * sizeof(int32_t));
        int32_t *g = (int32_t *)malloc(nb * sizeof(int32_t));
        int32_t *g2 = (int32_t *)malloc(nb * sizeof(int32_t));
        for (long p = 0; p < n; ++p) mk[p] = dq[p] - h_seed;
        or_recon(mk, dq, A, w, h, 8, g);
        for (long p = 0; p < n; ++p) mk[p] = g[p] - 1;
        or_recon(mk, g, A, w, h, 8, g2);
        for (long p = 0; p < n; ++p) rm[p] = (A[p] && g[p] - g2[p] > 0) ? 1 : 0;
        free(g2);
        free(g);
        free(mk);
    } else {
        for (long p = 0; p < n; ++p) rm[p] = (A[p] && seeds[p]) ? 1 : 0;
    }
    int32_t *S = (int32_t *)malloc(nb * sizeof(int32_t));
    or_ccl(rm, w, h, 8, S);
    if (seed_lab_out) memcpy(seed_lab_out, S, (size_t)n * sizeof(int32_t));

    /* lambda = recon_A(mu under Dq) */
    int32_t *mu = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *lam = (int32_t *)malloc(nb * sizeof(int32_t));
    for (long p = 0; p < n; ++p) mu[p] = S[p] > 0 ? dq[p] : INT32_MIN;
    or_recon(mu, dq, A, w, h, 8, lam);
    if (lambda_out) memcpy(lambda_out, lam, (size_t)n * sizeof(int32_t));

    /* flood, level by level */
    int32_t *lab = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *dist = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *levels = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc(nb * sizeof(int32_t));
    long nu = 0;
    for (long p = 0; p < n; ++p) {
        lab[p] = S[p];
        dist[p] = -1;
        if (A[p] && S[p] == 0 && lam[p] != INT32_MIN) levels[nu++] = lam[p];
    }
    qsort(levels, (size_t)nu, sizeof(int32_t), cmp_desc_i32);
    long nlev = 0;
    for (long i = 0; i < nu; ++i)
        if (nlev == 0 || levels[nlev - 1] != levels[i]) levels[nlev++] = levels[i];
    /* bucket the unlabelled pixels by level: order[] holds pixels grouped by level */
    {
        /* counting by binary search of the level index */
        long *start = (long *)calloc((size_t)nlev + 1, sizeof(long));
        int32_t *li = (int32_t *)malloc(nb * sizeof(int32_t));
        for (long p = 0; p < n; ++p) {
            li[p] = -1;
            if (!(A[p] && S[p] == 0 && lam[p] != INT32_MIN)) continue;
            long lo = 0, hi = nlev - 1;
            while (lo < hi) { /* levels strictly descending */
                long mid = (lo + hi) / 2;
                if (levels[mid] > lam[p])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            li[p] = (int32_t)lo;
            start[lo + 1]++;
        }
        for (long i = 0; i < nlev; ++i) start[i + 1] += start[i];
        long *fill = (long *)malloc(((size_t)nlev + 1) * sizeof(long));
        memcpy(fill, start, ((size_t)nlev + 1) * sizeof(long));
        for (long p = 0; p < n; ++p)
            if (li[p] >= 0) order[fill[li[p]]++] = (int32_t)p;
        for (long L = 0; L < nlev; ++L) {
            long b = start[L], e = start[L + 1];
            long qh = 0, qt = 0;
            /* layer 1: pixels of U_L with a neighbour labelled before level L
               (pixels reached during this level have dist >= 0 and are skipped) */
            for (long i = b; i < e; ++i) {
                int32_t p = order[i];
                int x = p % w, y = p / w;
                int32_t best = 0;
                for (int d = 0; d < 8; ++d) {
                    int qx = x + DX8[d], qy = y + DY8[d];
                    if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
                    long q = (long)qy * w + qx;
                    if (A[q] && lab[q] > 0 && dist[q] < 0 && (best == 0 || lab[q] < best)) best = lab[q];
                }
                if (best > 0) {
                    dist[p] = 1;
                    lab[p] = best;
                    queue[qt++] = p;
                }
            }
            /* layers 2, 3, ...: pixel takes the minimum label among its
               neighbours in the previous layer */
            while (qh < qt) {
                int32_t p = queue[qh++];
                int x = p % w, y = p / w;
                for (int d = 0; d < 8; ++d) {
                    int qx = x + DX8[d], qy = y + DY8[d];
                    if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
                    long q = (long)qy * w + qx;
                    if (li[q] != (int32_t)L) continue; /* not in U_L */
                    if (dist[q] < 0) {
                        dist[q] = dist[p] + 1;
                        lab[q] = lab[p];
                        queue[qt++] = (int32_t)q;
                    } else if (dist[q] == dist[p] + 1 && lab[p] < lab[q]) {
                        lab[q] = lab[p];
                    }
                }
            }
            /* pixels of this level are now "labelled before" the next level */
            for (long i = b; i < e; ++i) dist[order[i]] = -1;
        }
        free(fill);
        free(li);
        free(start);
    }
    /* leftovers (only with external seeds): ccl8 of the unlabelled set */
    {
        uint8_t *left = (uint8_t *)calloc(nb, 1);
        int any = 0;
        for (long p = 0; p < n; ++p)
            if (A[p] && lab[p] == 0) {
                left[p] = 1;
                any = 1;
            }
        if (any) {
            int32_t *ll = (int32_t *)malloc(nb * sizeof(int32_t));
            or_ccl(left, w, h, 8, ll);
            for (long p = 0; p < n; ++p)
                if (left[p]) lab[p] = ll[p];
            free(ll);
        }
        free(left);
    }
    if (flood_out) memcpy(flood_out, lab, (size_t)n * sizeof(int32_t));

    /* cut: drop p if an 8-neighbour carries a smaller nonzero label */
    uint8_t *M = (uint8_t *)malloc(nb);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            long p = (long)y * w + x;
            int32_t l = A[p] ? lab[p] : 0;
            int keep = l > 0;
            for (int d = 0; d < 8 && keep; ++d) {
                int qx = x + DX8[d], qy = y + DY8[d];
                if (qx < 0 || qy < 0 || qx >= w || qy >= h) continue;
                long q = (long)qy * w + qx;
                int32_t lq = A[q] ? lab[q] : 0;
                if (lq > 0 && lq < l) keep = 0;
            }
            M[p] = (uint8_t)keep;
        }
    or_ccl(M, w, h, 8, labels_out);
    if (mask_out) memcpy(mask_out, M, (size_t)n);
    if (dq_out) memcpy(dq_out, dq, (size_t)n * sizeof(int32_t));

    free(M);
    free(queue);
    free(levels);
    free(order);
    free(dist);
    free(lab);
    free(lam);
    free(mu);
    free(S);
    free(rm);
    free(dq);
    free(A);
}

/* ------------------------------------------------------------------------ */
/* Full plain pipeline from Hq                                              */
/* ------------------------------------------------------------------------ */

int or_segment_from_hq(const uint8_t *hq, int w, int h, int t_fg, int min_area, int max_area,
                       int h_seed, uint8_t *mask_out, int32_t *labels_out,
                       uint8_t *recon_out, uint8_t *f0_out, uint8_t *f_out, uint8_t *a_out) {
    long n = (long)w * h;
    size_t nb = (size_t)(n > 0 ? n : 1);
    int32_t *I = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *J = (int32_t *)malloc(nb * sizeof(int32_t));
    int32_t *R = (int32_t *)malloc(nb * sizeof(int32_t));
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            long p = (long)y * w + x;
            I[p] = hq[p];
            J[p] = (x == 0 || y == 0 || x == w - 1 || y == h - 1) ? hq[p] : 0;
        }
    or_recon(J, I, NULL, w, h, 8, R);
    uint8_t *F0 = (uint8_t *)malloc(nb);
    for (long p = 0; p < n; ++p) F0[p] = (I[p] - R[p] >= t_fg) ? 1 : 0;
    if (recon_out)
        for (long p = 0; p < n; ++p) recon_out[p] = (uint8_t)R[p];
    if (f0_out) memcpy(f0_out, F0, (size_t)n);
    uint8_t *F = (uint8_t *)malloc(nb);
    or_fill_holes(F0, w, h, 4, F);
    if (f_out) memcpy(f_out, F, (size_t)n);
    int32_t *L1 = (int32_t *)malloc(nb * sizeof(int32_t));
    or_ccl(F, w, h, 8, L1);
    uint8_t *A = (uint8_t *)malloc(nb);
    or_area_filter(L1, w, h, min_area, INT_MAX, L1, A);
    if (a_out) memcpy(a_out, A, (size_t)n);
    int32_t *L2 = (int32_t *)malloc(nb * sizeof(int32_t));
    or_watershed(A, NULL, h_seed, w, h, L2, NULL, NULL, NULL, NULL, NULL);
    int kept = or_area_filter(L2, w, h, min_area, max_area, labels_out, mask_out);
    free(L2);
    free(A);
    free(L1);
    free(F);
    free(F0);
    free(R);
    free(J);
    free(I);
    return kept;
}
