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

/* ------------------------------------------------------------------------
 * Feature computation (Sec. 5.1: shape and texture features per segmented
 * nucleus from per-nucleus histograms and co-occurrence matrices; Fig. 1:
 * 60-100 shape and texture features per object).  The paper lists no
 * feature; the set below is the reading, each from its textbook definition.
 *
 * Input: labels (int32, 0 = background, a nucleus = all pixels sharing one
 * positive label, label values <= w*h; labels as produced by the segmentation
 * are 1 + the row-major index of the nucleus' first pixel) and Hq (uint8).
 * Nuclei are reported in order of their first pixel in row-major order (for
 * such labels: increasing label).
 *
 * Per-nucleus counts (exact integers):
 *   area, bounding box, coordinate sums (x, y, x^2, y^2, xy);
 *   perimeter = number of pixel sides (4-neighbours) of the nucleus that face
 *     a pixel of another label or the outside of the tile;
 *   hist[v] = pixels with Hq = v;
 *   gradient magnitude g = floor(sqrt(gx^2 + gy^2)) of the 3x3 Sobel operator
 *     on Hq, pixels outside the tile replicating the nearest edge pixel;
 *     ghist[b] = pixels with min(g / OR_GRAD_BIN_WIDTH, OR_GRAD_BINS - 1) = b;
 *     sum g, sum g^2, max g;
 *   co-occurrence matrix C of Hq quantised to OR_GLCM_LEVELS levels
 *     (q = Hq / (256 / levels)) over the offsets (1,0), (1,1), (0,1), (-1,1)
 *     (0, 45, 90, 135 degrees, distance 1), pooled: every pair of pixels of
 *     the same nucleus at one of these offsets adds 1 to C[q1][q2] and 1 to
 *     C[q2][q1].
 * Features (FP64), in this order:
 *   shape: area; perimeter; centroid x, y; bbox width, height; extent =
 *     area / bbox area; equivalent diameter sqrt(4 area / pi); circularity
 *     4 pi area / perimeter^2; major and minor axis 4 sqrt(l1), 4 sqrt(l2) and
 *     eccentricity sqrt(1 - l2 / l1) with l1 >= l2 the eigenvalues of the
 *     second central moments (mu20, mu11; mu11, mu02) of the pixel set, each
 *     pixel a unit square (1/12 added to mu20 and mu02), mu20 =
 *     (A sum x^2 - (sum x)^2) / A^2 etc. (coordinates relative to the
 *     nucleus' first pixel; numerators exact in 128-bit integers, so
 *     w, h <= 32768); orientation 0.5 atan2(2 mu11,
 *     mu20 - mu02) (radians, y down);
 *   intensity of Hq: mean; standard deviation (population); min; max; median,
 *     25th and 75th percentile = the sorted values at 0-based ranks
 *     floor((A-1)/2), floor((A-1)/4), floor(3(A-1)/4); skewness m3 / m2^1.5
 *     and kurtosis m4 / m2^2 (central moments, 0 when m2 = 0); entropy
 *     -sum p log2 p and energy sum p^2 of the histogram; range max - min;
 *   gradient: mean g; standard deviation sqrt(A sum g^2 - (sum g)^2) / A;
 *     max g; entropy and energy of ghist; edge fraction = share of pixels with
 *     g >= OR_EDGE_THRESHOLD;
 *   Haralick texture of p = C / sum C (all 0 when sum C = 0), px its
 *     marginal (equal for rows and columns: C is symmetric), mu = sum i px(i),
 *     var = sum (i - mu)^2 px(i), p_{x+y}(k) and p_{x-y}(k) the sums of p over
 *     i + j = k and |i - j| = k: angular second moment sum p^2; contrast
 *     sum (i-j)^2 p; correlation sum (i-mu)(j-mu) p / var (1 when var = 0);
 *     variance var; homogeneity sum p / (1 + (i-j)^2); sum average
 *     sum k p_{x+y}; sum variance sum (k - sum average)^2 p_{x+y}; sum entropy;
 *     entropy -sum p log2 p; difference variance (about the mean of
 *     p_{x-y}); difference entropy; information measures of correlation
 *     IMC1 = (HXY - HXY1) / HX (0 when HX = 0) and IMC2 =
 *     sqrt(1 - exp(-2 max(HXY2 - HXY, 0))) with HX = -sum px log2 px,
 *     HXY1 = -sum p log2(px(i) px(j)), HXY2 = -sum px(i)px(j) log2(px(i)px(j));
 *     maximum probability; cluster shade sum (i + j - 2 mu)^3 p and cluster
 *     prominence sum (i + j - 2 mu)^4 p.
 * ------------------------------------------------------------------------ */
#define OR_GLCM_LEVELS 16
#define OR_GRAD_BINS 16
#define OR_GRAD_BIN_WIDTH 32
#define OR_EDGE_THRESHOLD 128
enum {
    OF_AREA, OF_PERIMETER, OF_CENTROID_X, OF_CENTROID_Y, OF_BBOX_W, OF_BBOX_H, OF_EXTENT, OF_EQUIV_DIAMETER,
    OF_CIRCULARITY, OF_MAJOR_AXIS, OF_MINOR_AXIS, OF_ECCENTRICITY, OF_ORIENTATION,
    OF_INT_MEAN, OF_INT_STD, OF_INT_MIN, OF_INT_MAX, OF_INT_MEDIAN, OF_INT_P25, OF_INT_P75, OF_INT_SKEWNESS,
    OF_INT_KURTOSIS, OF_INT_ENTROPY, OF_INT_ENERGY, OF_INT_RANGE,
    OF_GRAD_MEAN, OF_GRAD_STD, OF_GRAD_MAX, OF_GRAD_ENTROPY, OF_GRAD_ENERGY, OF_EDGE_FRACTION,
    OF_GLCM_ASM, OF_GLCM_CONTRAST, OF_GLCM_CORRELATION, OF_GLCM_VARIANCE, OF_GLCM_HOMOGENEITY,
    OF_GLCM_SUM_AVERAGE, OF_GLCM_SUM_VARIANCE, OF_GLCM_SUM_ENTROPY, OF_GLCM_ENTROPY, OF_GLCM_DIFF_VARIANCE,
    OF_GLCM_DIFF_ENTROPY, OF_GLCM_IMC1, OF_GLCM_IMC2, OF_GLCM_MAX_PROB, OF_GLCM_CLUSTER_SHADE,
    OF_GLCM_CLUSTER_PROMINENCE,
    OR_NFEAT
};
/* counts per nucleus: area, perimeter, x0, y0, x1, y1, hist[256], C[16][16]
   (row-major), ghist[16], sum g, sum g^2, max g */
#define OR_NCOUNT 537

/* Gradient magnitude of the feature stage at (x, y). */
int64_t or_sobel_mag(const uint8_t *hq, int w, int h, int x, int y);

/* Features of every nucleus (see above): labels_out[k], feats_out[k*OR_NFEAT +
 * i] for the first min(n, max_nuclei) nuclei; counts_out (nullable) receives
 * OR_NCOUNT counts per nucleus.  Returns the number of nuclei n. */
int or_features(const int32_t *labels, const uint8_t *hq, int w, int h, int max_nuclei, int32_t *labels_out,
                double *feats_out, int64_t *counts_out);

/* ------------------------------------------------------------------------
 * Pre-processing operations the paper lists beside the segmentation (Sec.
 * 5.1: Morphological Open, RBC detection, and the ReconToNuclei marker).
 * The paper defines none of them; the readings:
 *
 * Erosion / dilation (grey, uint8) with the flat disk B_r = {(dx, dy) :
 * dx^2 + dy^2 <= r^2}: out(p) = min (max) of in(p + d) over d in B_r with
 * p + d inside the tile (pixels outside the tile are ignored, i.e. padded
 * with 255 for erosion and 0 for dilation).  Opening = dilation of the
 * erosion, both with B_r.
 *
 * ReconToNuclei with a choice of marker: R = recon8(J under Hq) with
 * J = Hq on the 1-px tile frame and 0 inside (OR_MARKER_FRAME, the plain
 * pipeline's marker) or J = erosion of Hq by B_r (OR_MARKER_OPEN: opening
 * by reconstruction, so T is a top-hat by reconstruction);
 * F0 = [Hq - R >= t_fg].
 *
 * RBC detection: redness(p) = 2 R - G - B of the RGB pixel; the red blood
 * cell mask is every pixel of an 8-connected region of {redness >= t_weak}
 * that holds a pixel with redness >= t_strong (hysteresis thresholding, as a
 * binary reconstruction).
 * ------------------------------------------------------------------------ */
#define OR_MARKER_FRAME 0
#define OR_MARKER_OPEN 1
void or_erode(const uint8_t *in, int w, int h, int radius, uint8_t *out);
void or_dilate(const uint8_t *in, int w, int h, int radius, uint8_t *out);
void or_open(const uint8_t *in, int w, int h, int radius, uint8_t *out);
void or_recon_to_nuclei(const uint8_t *hq, int w, int h, int marker_mode, int radius, int t_fg, uint8_t *recon_out,
                        uint8_t *f0_out);
void or_rbc_detect(const uint8_t *rgb, int w, int h, int t_strong, int t_weak, uint8_t *mask_out);

/* ------------------------------------------------------------------------
 * Cross-tile stitching with ghost cells (Sec. 3.4: partitions of a data
 * region are extended with ghost cells from their neighbours).  The slide
 * (W x H, Hq given) is cut into tile x tile cores in row-major order (the
 * last row and column ragged); each core is extended by `halo` pixels on
 * every side, clipped at the slide edge, and the extended region is
 * segmented on its own (or_segment_from_hq with the given parameters).  A
 * core owns the nuclei of its extended result whose first pixel (the root of
 * the label) lies inside the core; each owned nucleus is written into the
 * slide label map with the slide label 1 + (slide row-major index of its
 * first pixel).  Where owned nuclei of two cores cover the same pixel the
 * smaller slide label is kept.  mask_out (nullable) = labels_out != 0.
 * Returns the number of owned nuclei.
 * ------------------------------------------------------------------------ */
int or_stitch_from_hq(const uint8_t *hq, int W, int H, int tile, int halo, int t_fg, int min_area, int max_area,
                      int h_seed, int32_t *labels_out, uint8_t *mask_out);

#ifdef __cplusplus
}
#endif
#endif
