/*
 * rt_oracle.h -- plain, slow, single-threaded CPU oracle for per-tile nucleus
 * segmentation (the segmentation stage of the paper's example application,
 * Sec. 5.1 "Example Application").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library, and the GPU
 * library never calls it.
 *
 * The paper names the operations (colour deconvolution, ReconToNuclei,
 * FillHoles, AreaThreshold, BWLabel, Pre-Watershed, Watershed; Sec. 5.1 and
 * the PATS discussion in Sec. 3.2.1) but defines none of them.  Every function
 * here computes the textbook definition written out in its comment; where the
 * paper is silent the reading is stated.  Images are row-major, dense
 * (pitch == width), pixel (x, y) at index y*w + x.
 *
 * Connectivity: 8 = the 3x3 neighbourhood, 4 = the cross.
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define OR_DQ_MAX 65535

/* Colour deconvolution (Sec. 5.1; Ruifrok-Johnston stain separation).
 * stain_rows: 3 stain optical-density row vectors (H, E, third).  Each row is
 * L2-normalised; a zero third row is replaced by normalize(H x E).  With
 * M = [H; E; third] the optical density of a pixel is OD = c * M, so the
 * hematoxylin concentration is c_H = sum_k OD_k * inv(M)[k][0].
 * OD_k = -ln((I_k + 1) / 256).  c_H is summed as (R-term + G-term) + B-term
 * in FP64 without contraction; Hq = clamp(floor(c_H * scale + 0.5), 0, 255).
 * rgb is interleaved RGB bytes, 3*w*h.  cH_out (nullable) receives c_H.
 * Returns 0, or -1 if the stain matrix is singular. */
int or_deconv(const uint8_t *rgb, int w, int h, const double stain_rows[9], double scale,
              double *cH_out, uint8_t *hq_out);

/* c_H for one optical-density vector (used by the closed-form pins). */
int or_deconv_od(const double stain_rows[9], const double od[3], double *cH);

/* Grayscale reconstruction by dilation (Vincent 1993), int32 values.
 * out(p) = max over paths p0..pn = p inside the graph of
 *          min(min(marker,mask)(p0), mask(p1), ..., mask(pn)),
 * computed as a widest-path search with a binary max-heap.  Graph nodes are the
 * pixels with domain != 0 (all pixels if domain is NULL); edges join
 * conn-neighbours that are both nodes.  Pixels outside the domain get
 * min(marker, mask) and take no part in the propagation. */
void or_recon(const int32_t *marker, const int32_t *mask, const uint8_t *domain, int w, int h,
              int conn, int32_t *out);

/* Hole filling: a 0-pixel stays 0 iff it is bg_conn-connected through 0-pixels
 * to a 0-pixel on the tile frame; every other pixel becomes 1. */
void or_fill_holes(const uint8_t *in, int w, int h, int bg_conn, uint8_t *out);

/* Connected-component labelling of nonzero pixels.  label(p) = 1 + the
 * smallest row-major index y*w + x in the component of p; 0 = background.
 * Returns the number of components. */
int or_ccl(const uint8_t *mask, int w, int h, int conn, int32_t *labels);

/* Area threshold: components (by label value) with min_area <= area <= max_area
 * keep their label, others become 0.  mask_out (nullable) = labels_out != 0.
 * Returns the number of kept components. */
int or_area_filter(const int32_t *labels_in, int w, int h, int min_area, int max_area,
                   int32_t *labels_out, uint8_t *mask_out);

/* Exact squared Euclidean distance transform.  For fg(p) != 0:
 * d2(p) = min over in-tile q with fg(q) == 0 of (xp-xq)^2 + (yp-yq)^2;
 * 0 for background; -1 for every pixel if the tile has no 0-pixel.
 * Separable exact method (column distances, then the lower envelope of
 * parabolas per row; Felzenszwalb-Huttenlocher / Meijster et al.). */
void or_edt_sq(const uint8_t *fg, int w, int h, int64_t *d2);

/* floor(sqrt(n)) for n >= 0, exact. */
int64_t or_isqrt(int64_t n);

/* Quantised distance Dq(p) = floor(sqrt(4 d2(p))) (half-pixel units) on fg,
 * 0 on background, OR_DQ_MAX on fg when the tile has no 0-pixel. */
void or_dq(const uint8_t *fg, int w, int h, int32_t *dq);

/* Watershed split of the foreground (Pre-Watershed + Watershed, Sec. 5.1).
 *   Dq as above on A = fg.
 *   Seeds (seeds == NULL): g = recon_A(Dq - h_seed under Dq) (h-maxima);
 *     RM = { p in A : g(p) - recon_A(g - 1 under g)(p) > 0 } (regional maxima);
 *     seed labels S = ccl8(RM).  Otherwise S = ccl8(seeds AND A).
 *   lambda = recon_A(mu under Dq), mu = Dq on seed pixels, INT32_MIN elsewhere.
 *   Flood: levels L from max lambda down; U_L = unlabelled pixels with
 *     lambda = L; a breadth-first search from every pixel labelled so far into
 *     U_L through 8-neighbours inside U_L; a pixel reached in layer k takes the
 *     smallest label among its layer-(k-1) neighbours.  Pixels never reached
 *     (only with external seeds) get ccl8 labels of the leftover set.
 *   Cut: M(p) = 1 iff label(p) > 0 and no 8-neighbour q has 0 < label(q) < label(p).
 *   labels_out = ccl8(M), mask_out = M.
 * Optional intermediates (nullable): dq, seed labels, lambda, flood labels. */
void or_watershed(const uint8_t *fg, const uint8_t *seeds, int h_seed, int w, int h,
                  int32_t *labels_out, uint8_t *mask_out,
                  int32_t *dq_out, int32_t *seed_lab_out, int32_t *lambda_out, int32_t *flood_out);

/* Full plain segmentation from the quantised hematoxylin channel Hq:
 *   R = recon8(J under Hq), J = Hq on the 1-px tile frame, 0 inside;
 *   F0 = [Hq - R >= t_fg]; F = fill_holes(F0, 4); L1 = ccl8(F);
 *   A = components of L1 with area >= min_area;
 *   watershed(A, h_seed); labels = area filter [min_area, max_area] of its ccl8.
 * Optional intermediates (nullable): R, F0, F, A.  Returns n_objects. */
int or_segment_from_hq(const uint8_t *hq, int w, int h, int t_fg, int min_area, int max_area,
                       int h_seed, uint8_t *mask_out, int32_t *labels_out,
                       uint8_t *recon_out, uint8_t *f0_out, uint8_t *f_out, uint8_t *a_out);

#ifdef __cplusplus
}
#endif
#endif
