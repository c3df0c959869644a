/*
 * rtseg.h -- C ABI of the MI355X (gfx950) per-tile nucleus segmentation
 * library librtseg.so.
 *
 * What is computed: the segmentation stage of the example application of
 * Teodoro et al., "Region Templates" (Sec. 5.1, Example Application): a stage
 * receives an RGB tile and produces a mask of segmented nuclei (the
 * RGB-in / Mask-out stage boundary of Fig. 8b, Sec. 3.4).  The paper names the
 * operations -- colour deconvolution, ReconToNuclei, FillHoles,
 * AreaThreshold, BWLabel (union-find CCL), Pre-Watershed and Watershed
 * (Sec. 5.1; the operation list of the PATS discussion, Sec. 3.2.1) -- but
 * defines none of them; the definitions each entry point implements are
 * stated below.
 *
 * Conventions for every entry point
 *   - Image pointers are DEVICE pointers (e.g. PyTorch CUDA/HIP tensors).  The
 *     caller owns every buffer; the library never frees caller memory.
 *   - Images are row-major.  Pixel (x, y) of an image with pitch P (in
 *     elements, P >= w; for RGB the pitch is in bytes, >= 3*w) is element
 *     y*P + x.  Label values use the WIDTH, never the pitch:
 *     label = 1 + y*w + x of the component's first pixel in row-major order.
 *   - Sizes: w*h <= 2^31 - 2; rt_watershed, rt_segment_tile and
 *     rt_segment_batch, which pack a tile index and a pixel id into 32 bits,
 *     take w*h <= 2^25 - 2 (up to 5792 x 5792).
 *   - Connectivity 8 = the 3x3 neighbourhood, 4 = the cross.  Only in-tile
 *     pixels exist (no virtual padding beyond the tile edge).
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *     is the default stream) unless noted.  A few calls must read a small
 *     device counter to decide how many propagation rounds to launch; they
 *     synchronise `stream` for that and say so.
 *   - Scratch memory comes from the context and is reused by later calls on
 *     the same context: one context must not be used by two host threads (or
 *     two streams) at once.
 *   - Return value 0 = RT_OK; a negative value is an error code and
 *     rt_last_error() returns a thread-local message.  Asynchronous kernel
 *     faults surface on a later call or in rt_sync().
 */
#ifndef RTSEG_H
#define RTSEG_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define RT_OK 0
#define RT_EINVAL (-1)       /* bad argument: null pointer, w/h <= 0, pitch < w, too many pixels, bad conn/dtype, min > max */
#define RT_ENOMEM (-2)       /* scratch allocation failed */
#define RT_EDEVICE (-3)      /* HIP runtime error */
#define RT_EUNSUPPORTED (-4) /* valid request the library does not implement */

#define RT_U8 1
#define RT_I32 2

#define RT_DQ_MAX 65535

typedef struct rt_ctx rt_ctx;

/* Creates a context on HIP device `device`.  *out receives the handle. */
int rt_ctx_create(int device, rt_ctx **out);
/* Frees the context's scratch memory (synchronises the device first). */
int rt_ctx_destroy(rt_ctx *ctx);
/* Message of the last error on the calling thread ("" if none). */
const char *rt_last_error(void);
/* Waits for `stream`, then reports any pending asynchronous device error. */
int rt_sync(rt_ctx *ctx, void *stream);

/*
 * Colour deconvolution (Sec. 5.1; Ruifrok-Johnston stain separation).
 * stain_rows: 3 optical-density row vectors (hematoxylin, eosin, third); each
 * is L2-normalised and a zero third row is replaced by normalize(H x E).  With
 * M = [H; E; third], OD = c * M, so c_H = sum_k OD_k * inv(M)[k][0], with
 * OD_k = -ln((I_k + 1) / 256).  The sum is evaluated in FP64 as
 * (R-term + G-term) + B-term without contraction, and
 * hq = clamp(floor(c_H * hq_scale + 0.5), 0, 255).
 * rgb: interleaved RGB bytes, row pitch rgb_pitch_bytes.  cH_out (nullable):
 * float c_H, pitch cH_pitch elements.  hq_out: uint8, pitch hq_pitch.
 * Errors: RT_EINVAL for a singular stain matrix or bad sizes.
 */
int rt_deconv(rt_ctx *ctx, const uint8_t *rgb, int64_t rgb_pitch_bytes, int32_t w, int32_t h,
              const double stain_rows[9], double hq_scale, float *cH_out, int64_t cH_pitch,
              uint8_t *hq_out, int64_t hq_pitch, void *stream);

/*
 * Grayscale reconstruction by dilation (the IWPP operation behind
 * ReconToNuclei, Sec. 5.1).  dtype RT_U8 (uint8 images) or RT_I32 (int32).
 * out(p) = max over paths p0..pn = p inside the graph of
 *          min(min(marker,mask)(p0), mask(p1), ..., mask(pn)).
 * Graph nodes are the pixels with domain != 0 (all pixels if domain is NULL);
 * pixels outside the domain get min(marker, mask) and take no part.
 * marker, mask, out and domain share `pitch` (elements).  out may alias
 * marker.  conn is 4 or 8.  Synchronises `stream` between propagation rounds.
 */
int rt_morph_recon(rt_ctx *ctx, int dtype, const void *marker, const void *mask, void *out,
                   const uint8_t *domain, int32_t w, int32_t h, int64_t pitch, int conn, void *stream);

/*
 * FillHoles (Sec. 5.1): a 0-pixel of `in` stays 0 iff it is
 * bg_conn-connected through 0-pixels to a 0-pixel on the tile frame; every
 * other pixel becomes 1.  bg_conn is 4 (default) or 8.  out may alias in.
 */
int rt_fill_holes(rt_ctx *ctx, const uint8_t *in, uint8_t *out, int32_t w, int32_t h, int64_t pitch,
                  int bg_conn, void *stream);

/*
 * BWLabel (Sec. 5.1; union-find forest, merge, flatten).  Labels the nonzero
 * pixels of `mask`: label(p) = 1 + min{ y*w + x : (x, y) in the component of p },
 * 0 for background.  labels is int32 with pitch `pitch`.  n_out_dev (nullable,
 * device int32) receives the number of components.
 */
int rt_ccl(rt_ctx *ctx, const uint8_t *mask, int32_t *labels, int32_t w, int32_t h, int64_t pitch, int conn,
           int32_t *n_out_dev, void *stream);

/*
 * rt_ccl without allocation, for callers that cannot allocate memory during a
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, definition and output as rt_ccl.  Its
 * scratch (an argument record, the union-find array of 4 (w*h + 1) bytes,
 * a border table of 1 KB per 64 x 64 tile and, when n_out_dev is given, a
 * component list) lives in one fixed device
 * array of RT_NOALLOC_SCRATCH_BYTES bytes, which every device the library
 * runs on holds until the process ends; the array's device address is
 * looked up when a context is first created on the device.  The call makes
 * no hipMalloc, hipFree, pinned-memory or other allocating call and no
 * memset (counters are cleared by a kernel).
 * Limits: w*h <= RT_NOALLOC_MAX_PIXELS (e.g. 2048 x 2048); larger images
 * return RT_EINVAL with a message.  Every call on one device shares the
 * array: calls that overlap on one device (two streams, two host threads,
 * two contexts) race and must be serialised by the caller.
 */
#define RT_NOALLOC_SCRATCH_BYTES (32 << 20)
#define RT_NOALLOC_MAX_PIXELS (1 << 22)
int rt_ccl_noalloc(rt_ctx *ctx, const uint8_t *mask, int32_t *labels, int32_t w, int32_t h, int64_t pitch,
                   int conn, int32_t *n_out_dev, void *stream);

/*
 * AreaThreshold (Sec. 5.1): a component (pixels sharing one positive label)
 * with min_area <= area <= max_area keeps its label; other pixels become 0.
 * Labels must be < w*h + 1 (e.g. produced by rt_ccl).  mask_out (nullable,
 * uint8) = labels_out != 0.  labels_out may alias labels_in.
 */
int rt_area_filter(rt_ctx *ctx, const int32_t *labels_in, int32_t *labels_out, uint8_t *mask_out,
                   int32_t w, int32_t h, int64_t pitch, int32_t min_area, int32_t max_area, void *stream);

/*
 * Pre-Watershed + Watershed (Sec. 5.1) on the foreground A = (fg != 0):
 *   Dq = floor(sqrt(4 d2)), d2 = squared distance to the nearest in-tile
 *        0-pixel of A (RT_DQ_MAX if A has no 0-pixel);
 *   seeds (seeds == NULL): regional maxima of the h-maxima transform
 *        g = recon_A(Dq - h_seed under Dq), labelled by 8-connected CCL;
 *        otherwise the 8-connected components of (seeds != 0) AND A;
 *   lambda = recon_A(Dq on seed pixels under Dq);
 *   flood from high to low lambda: a breadth-first search into each level set
 *        from everything labelled so far, where a pixel takes the smallest
 *        label among its neighbours in the previous search layer; pixels never
 *        reached (possible only with external seeds) are labelled by CCL;
 *   cut: p is kept iff no 8-neighbour carries a smaller nonzero label;
 *   labels_out = 8-connected CCL of the kept pixels, mask_out = kept pixels.
 * fg, seeds, mask_out (uint8) and labels_out (int32) share `pitch`.
 */
int rt_watershed(rt_ctx *ctx, const uint8_t *fg, const uint8_t *seeds, int32_t h_seed, int32_t *labels_out,
                 uint8_t *mask_out, int32_t w, int32_t h, int64_t pitch, void *stream);

/* Parameters of the whole plain pipeline.  size must be sizeof(rt_seg_params). */
typedef struct {
    uint32_t size;
    double stain_rows[9]; /* H, E, third (zero row = H x E) optical-density vectors */
    double hq_scale;      /* 85.0 */
    int32_t t_fg;         /* top-hat threshold, 16 */
    int32_t min_area;     /* 20 */
    int32_t max_area;     /* 1000 */
    int32_t h_seed;       /* 3 (half-pixel units) */
    int32_t conn;         /* foreground connectivity, 8 */
} rt_seg_params;

/* Fills p with the defaults above (Ruifrok-Johnston H&E vectors). */
void rt_seg_params_default(rt_seg_params *p);

/*
 * Segmentation stage of one tile (RGB in, mask + labels out):
 *   Hq = deconvolution; R = recon8(J under Hq) with J = Hq on the 1-px tile
 *   frame and 0 inside (ReconToNuclei); F0 = [Hq - R >= t_fg];
 *   F = FillHoles(F0, 4); L1 = CCL8(F); A = components of L1 with
 *   area >= min_area; watershed(A, h_seed); labels = components of its
 *   CCL8 with min_area <= area <= max_area; mask = labels != 0.
 * mask_out (uint8) and labels_out (int32) share out_pitch.  n_objects_dev
 * (nullable, device int32) receives the number of kept objects.  hq_out
 * (nullable, uint8, pitch out_pitch) receives the quantised hematoxylin
 * channel.  Synchronises `stream` between reconstruction rounds.
 */
int rt_segment_tile(rt_ctx *ctx, const uint8_t *rgb, int64_t rgb_pitch_bytes, int32_t w, int32_t h,
                    const rt_seg_params *params, uint8_t *mask_out, int32_t *labels_out, int64_t out_pitch,
                    int32_t *n_objects_dev, uint8_t *hq_out, void *stream);

/*
 * The same segmentation stage on a batch of independent tiles of any sizes
 * (the data-parallel execution of many tiles of an image, Sec. 3.2 and
 * Sec. 5.1): each tile's outputs equal those of rt_segment_tile on that tile
 * alone.  The tiles are processed in launch groups of up to 64; each stage of
 * a group is one kernel launch over all its tiles, so small and ragged tiles
 * share the device instead of running one after another.  Every descriptor
 * follows rt_segment_tile's argument rules; outputs of different tiles must
 * not overlap.  Synchronises `stream` between reconstruction rounds.
 * Errors: RT_EINVAL (checked for every tile before any work starts).
 */
typedef struct {
    const uint8_t *rgb;      /* device, interleaved RGB */
    int64_t rgb_pitch_bytes; /* >= 3*w */
    int32_t w, h;            /* w*h <= 2^25 - 2 */
    uint8_t *mask_out;       /* device, pitch out_pitch */
    int32_t *labels_out;     /* device, pitch out_pitch */
    int64_t out_pitch;       /* elements, >= w */
    int32_t *n_objects_dev;  /* nullable device int32 */
    uint8_t *hq_out;         /* nullable device uint8; needs out_pitch == w */
    uint8_t *fg_out;         /* nullable device uint8, pitch out_pitch: the foreground A after the
                                first area threshold (the watershed's input), 0/1 */
    uint8_t *seeds_out;      /* nullable (given iff fg_out is): the watershed seeds (regional
                                maxima of the h-maxima transform of Dq) inside A, 0/1 */
} rt_tile_desc;
int rt_segment_batch(rt_ctx *ctx, int32_t n, const rt_tile_desc *tiles, const rt_seg_params *params, void *stream);

/*
 * Cross-tile stitching with ghost cells (Sec. 3.4: partitions of a data
 * region are extended by ghost cells from their neighbours, so that objects
 * cut by a partition border are processed whole).  The slide (W x H RGB,
 * device) is cut into tile x tile cores in row-major order (the last row and
 * column ragged); each core is extended by `halo` pixels on every side
 * (clipped at the slide edge) and the extended tile is segmented exactly as
 * rt_segment_tile would (launch groups of up to 64 extended tiles, read in
 * place from the slide).  A core owns the nuclei of its extended result whose
 * first pixel (the root of the label) lies inside the core; each owned
 * nucleus is written into labels_out with its slide label 1 + (slide
 * row-major index of its first pixel), the smaller slide label winning where
 * nuclei of two cores cover one pixel.  mask_out (nullable) = labels_out != 0;
 * hq_out (nullable) receives the slide's quantised hematoxylin channel;
 * n_objects_dev (nullable) the number of owned nuclei.  labels, mask and Hq
 * share out_pitch.  (tile + 2 halo)^2 <= 2^25 - 2.  Synchronises `stream`
 * between reconstruction rounds unless the recon_async knob is set.
 */
int rt_segment_slide(rt_ctx *ctx, const uint8_t *rgb, int64_t rgb_pitch_bytes, int32_t W, int32_t H, int32_t tile,
                     int32_t halo, const rt_seg_params *params, int32_t *labels_out, uint8_t *mask_out,
                     int64_t out_pitch, uint8_t *hq_out, int32_t *n_objects_dev, void *stream);

/*
 * Host-resident tile streams (the prefetching and asynchronous copies of
 * Sec. 3.2.1, measured as "Pref." in Sec. 5.5): segments n tiles that live in
 * HOST memory and writes the results to host memory, overlapping the upload
 * of tile k+1 and the download of tile k-1 with the computation of tile k
 * (three device slots; copies on two streams of the context, computation on
 * `stream`, ordered by events).  Each tile is computed exactly as
 * rt_segment_tile would compute it.  Host buffers should be pinned
 * (hipHostMalloc) for the copies to overlap; pageable memory works but its
 * copies do not overlap.  mask / labels / n_objects may each be NULL (not
 * downloaded).  depth 1 runs upload, computation and download one after the
 * other (no overlap), 2 or 3 overlaps them.  The call returns when every
 * result is in host memory (it synchronises the context's streams).
 * Device scratch: depth slots of 8 bytes per pixel of the largest tile, plus
 * rt_segment_tile's own.
 * Errors: RT_EINVAL (checked for every tile before any work starts).
 */
typedef struct {
    const uint8_t *rgb;      /* host, interleaved RGB */
    int64_t rgb_pitch_bytes; /* >= 3*w */
    int32_t w, h;            /* w*h <= 2^25 - 2 */
    uint8_t *mask;           /* nullable host uint8, pitch out_pitch */
    int32_t *labels;         /* nullable host int32, pitch out_pitch */
    int64_t out_pitch;       /* elements, >= w */
    int32_t *n_objects;      /* nullable host int32 */
} rt_host_tile;
int rt_segment_host_stream(rt_ctx *ctx, int32_t n, const rt_host_tile *tiles, const rt_seg_params *params,
                           int32_t depth, void *stream);

/*
 * Tuning knobs of a context (set by the autotuner; results never depend on
 * them, only speed does):
 *   "recon_levels"      0..8  threshold levels of the frame-connectivity lower
 *                             bound that starts ReconToNuclei (0 = start from
 *                             the frame marker alone); default 2
 *   "recon_level_mode"  0|1   choice of those levels from the Hq histogram:
 *                             0: the values at which the share of pixels at
 *                             or above falls below 0.75 .. 0.33 (evenly
 *                             spaced); 1: consecutive values v0 - n + 2 ..
 *                             v0 + 1, v0 the highest value with a share of at
 *                             least recon_level_frac / 1000 at or above it
 *                             (n = 1: v0); default 1
 *   "recon_level_frac"  1..999 per mille for recon_level_mode 1; default 500
 *   "recon_round_batch" 1..64 propagation rounds launched between two reads of
 *                             the worklist counter; default 8
 *   "recon_max_sweeps"  1..1024 in-tile sweeps before a tile re-queues itself;
 *                             default 64
 *   "recon_mode"        0..2  0: reconstruction in rounds (all queued tiles per
 *                             launch, host checks between round batches);
 *                             1: one persistent work-queue launch (waves take
 *                             tiles from a device queue and push neighbours;
 *                             if a wave waits longer than 2 ms the remaining
 *                             work runs in rounds); 2: recon_queue_after
 *                             rounds as launches, then the work queue seeded
 *                             with the tiles they left queued; default 0
 *   "recon_queue_after" 1..64 rounds before the work queue in mode 2; default 2
 *   "recon_async"       0|1   1: the segmentation entry points never read the
 *                             worklist on the host: they launch
 *                             "recon_async_rounds" rounds, then one workgroup
 *                             finishes any rounds still needed on the device
 *                             (tile by tile; slow only for inputs that need
 *                             many more rounds), so rt_segment_tile /
 *                             rt_segment_batch return without waiting for the
 *                             device (beyond the reuse of the context's 4
 *                             argument-upload buffers) and with "graph" the
 *                             whole call is two graph launches; recon_mode
 *                             must be 0; default 0
 *   "recon_async_rounds" 1..256 launched rounds in async mode; default 16
 *   "objects_streams"   0|1   1: the three LDS per-object classes run side by
 *                             side on the call's stream and two side streams;
 *                             0: one after the other on the call's stream;
 *                             default 1
 *   (read only) "recon_host_reads": worklist counters read by the host so far
 *   "objects_path"      0     routing of components to the per-object kernels:
 *                             crops <= 32^2 and <= 64^2 to the register-scan
 *                             classes, up to 9312 px to the LDS class, larger
 *                             to global memory.  The values 1 (no 64^2 class)
 *                             and 2 (every crop to the LDS class) are switched
 *                             off and return RT_EUNSUPPORTED
 *   "graph"             0|1   rt_segment_tile / rt_segment_batch replay the
 *                             launch sequence from captured HIP graphs (cached
 *                             per tile-size list, up to 4); default 0.  The
 *                             first graph holds "graph_rounds" reconstruction
 *                             rounds; if tiles are still queued after them the
 *                             remaining rounds run as ordinary launches before
 *                             the second graph.  Ignored while stage timing is on.
 *   "graph_rounds"      1..4096; default 24
 * Read-only (rt_get_knob): "graph_captures", "graph_replays" (counts since
 * the context was created), "last_rounds" (reconstruction rounds of the last
 * segmentation call), "device" (the context's HIP device).
 * Errors: RT_EINVAL for an unknown name or a value out of range.
 */
int rt_set_knob(rt_ctx *ctx, const char *name, int value);
int rt_get_knob(rt_ctx *ctx, const char *name, int *value);

/*
 * Pre-processing operations listed beside the segmentation (Sec. 5.1:
 * Morphological Open, RBC detection; the PATS discussion of Sec. 5.5 names
 * them among the low-speedup operations).  The paper defines none of them.
 *
 * rt_morph: grey erosion (op RT_ERODE), dilation (RT_DILATE) or opening
 * (RT_OPEN = dilation of the erosion) of a uint8 image by the flat disk
 * B_r = {(dx, dy) : dx^2 + dy^2 <= r^2}, 0 <= r <= RT_MORPH_MAX_RADIUS:
 * out(p) = min (max) of in(p + d) over d in B_r with p + d inside the image
 * (pixels outside are ignored).  in and out are uint8 with their own
 * pitches and must not overlap.  RT_OPEN takes w*h bytes of scratch.
 */
#define RT_ERODE 0
#define RT_DILATE 1
#define RT_OPEN 2
#define RT_MORPH_MAX_RADIUS 32
int rt_morph(rt_ctx *ctx, int op, const uint8_t *in, int64_t in_pitch, uint8_t *out, int64_t out_pitch, int32_t w,
             int32_t h, int32_t radius, void *stream);

/*
 * ReconToNuclei with a choice of marker: R = reconstruction by dilation
 * (8-connected) of the marker J under Hq, with J = Hq on the one-pixel tile
 * frame and 0 inside (RT_MARKER_FRAME, the marker of rt_segment_tile) or
 * J = erosion of Hq by B_radius (RT_MARKER_OPEN: opening by reconstruction,
 * so Hq - R is a top-hat by reconstruction); F0 = [Hq - R >= t_fg].
 * hq, r_out (nullable: R is then kept in scratch) and f0_out share `pitch`.
 * Synchronises `stream` between reconstruction rounds, like rt_morph_recon.
 */
#define RT_MARKER_FRAME 0
#define RT_MARKER_OPEN 1
int rt_recon_to_nuclei(rt_ctx *ctx, const uint8_t *hq, uint8_t *r_out, uint8_t *f0_out, int32_t w, int32_t h,
                       int64_t pitch, int marker, int32_t radius, int32_t t_fg, void *stream);

/*
 * RBC detection: redness(p) = 2 R - G - B of the interleaved RGB pixel; the
 * red blood cell mask (uint8 0/1, pitch out_pitch) holds every pixel of an
 * 8-connected region of {redness >= t_weak} that contains a pixel with
 * redness >= t_strong (hysteresis thresholding, computed as a binary
 * reconstruction).  t_weak <= t_strong.  Synchronises `stream` between
 * reconstruction rounds.  Scratch: out_pitch * h bytes.
 */
int rt_rbc_detect(rt_ctx *ctx, const uint8_t *rgb, int64_t rgb_pitch_bytes, int32_t w, int32_t h, int32_t t_strong,
                  int32_t t_weak, uint8_t *mask_out, int64_t out_pitch, void *stream);

/*
 * Feature computation (Sec. 5.1: shape and texture features of every
 * segmented nucleus, computed in two steps -- one block per nucleus bounding
 * box builds the nucleus' histograms and co-occurrence matrix, then one
 * thread per nucleus computes the features; Fig. 1: a vector of shape and
 * texture features per object).  The paper lists no feature; the set is:
 *
 * Input: labels (int32, pitch lab_pitch; 0 = background; a nucleus is every
 * pixel carrying one positive label, whose value is 1 + the row-major index
 * y*w + x of the nucleus' first pixel -- the labels rt_segment_tile, rt_ccl
 * and rt_watershed produce) and Hq (uint8, pitch hq_pitch).  Nuclei are
 * numbered in increasing label order; the first min(n, max_nuclei) are
 * written.  Other label values are ignored (memory-safe, unspecified
 * features).  w, h <= 32768.
 * Per-nucleus counts (exact): area; bounding box; perimeter = pixel sides of
 * the nucleus (4-neighbours) that face another label or the outside of the
 * tile; hist[v] = pixels with Hq = v; Sobel gradient g = floor(sqrt(gx^2 +
 * gy^2)) of Hq (3 x 3 kernels with weights 1, 2, 1; pixels outside the tile
 * replicate the nearest edge pixel) with its histogram ghist[min(g / 32, 15)],
 * sum, sum of squares and maximum; co-occurrence matrix C of the grey levels
 * Hq / 16 (16 levels) over the offsets (1,0), (1,1), (0,1), (-1,1): every
 * pair of pixels of the nucleus at one of them adds 1 to C[q1][q2] and to
 * C[q2][q1].
 * Features (FP64, RT_NFEAT per nucleus, in this order):
 *    0 area  1 perimeter  2 centroid x  3 centroid y  4 bbox width
 *    5 bbox height  6 extent (area / bbox area)  7 equivalent diameter
 *    sqrt(4 area / pi)  8 circularity 4 pi area / perimeter^2
 *    9 major axis 4 sqrt(l1)  10 minor axis 4 sqrt(l2)  11 eccentricity
 *    sqrt(1 - l2 / l1)  12 orientation 0.5 atan2(2 mu11, mu20 - mu02)
 *    (radians, y down) -- l1 >= l2 the eigenvalues of the second central
 *    moments of the pixel set with each pixel a unit square (1/12 added to
 *    mu20 and mu02); A^2 mu20 = A sum x^2 - (sum x)^2 etc. exact in 128 bits;
 *   13 mean  14 standard deviation  15 min  16 max  17 median  18 25th and
 *   19 75th percentile of Hq (the sorted values at 0-based ranks
 *   floor((A-1)/2), floor((A-1)/4), floor(3(A-1)/4))  20 skewness m3/m2^1.5
 *   21 kurtosis m4/m2^2 (0 when m2 = 0)  22 entropy -sum p log2 p and
 *   23 energy sum p^2 of the Hq histogram  24 range max - min;
 *   25 mean g  26 standard deviation of g  27 max g  28 entropy and
 *   29 energy of ghist  30 share of pixels with g >= 128;
 *   Haralick features of p = C / sum C (all 0 when sum C = 0; px the
 *   marginal, mu = sum i px, var = sum (i-mu)^2 px, p_{x+y}, p_{x-y} the
 *   sums over i+j = k and |i-j| = k): 31 angular second moment
 *   32 contrast  33 correlation (1 when var = 0)  34 variance
 *   35 homogeneity sum p / (1 + (i-j)^2)  36 sum average  37 sum variance
 *   38 sum entropy  39 entropy  40 difference variance  41 difference entropy
 *   42 IMC1 = (HXY - HXY1) / HX (0 when HX = 0)  43 IMC2 =
 *   sqrt(1 - exp(-2 max(HXY2 - HXY, 0)))  44 maximum probability
 *   45 cluster shade sum (i+j-2mu)^3 p  46 cluster prominence
 *   sum (i+j-2mu)^4 p.  Logarithms base 2.
 * Outputs (device memory owned by the caller): labels_out[max_nuclei] (the
 * nuclei's labels), feats_out[max_nuclei * RT_NFEAT], counts_out (nullable,
 * int64, max_nuclei * RT_FEAT_NCOUNT: area, perimeter, x0, y0, x1, y1,
 * hist[256], C[16][16] row-major, ghist[16], sum g, sum g^2, max g) and
 * n_out_dev (nullable, int32: the number of nuclei, also beyond max_nuclei).
 * Scratch: 4 (w*h + h + 1) bytes plus about 2.2 KB per nucleus.
 */
#define RT_NFEAT 47
#define RT_FEAT_NCOUNT 537
#define RT_FEAT_GLCM_LEVELS 16
#define RT_FEAT_GRAD_BINS 16
#define RT_FEAT_GRAD_BIN_WIDTH 32
#define RT_FEAT_EDGE_THRESHOLD 128
int rt_features(rt_ctx *ctx, const int32_t *labels, int64_t lab_pitch, const uint8_t *hq, int64_t hq_pitch,
                int32_t w, int32_t h, int32_t max_nuclei, int32_t *labels_out, double *feats_out,
                int64_t *counts_out, int32_t *n_out_dev, void *stream);

/*
 * Stage timing, for benchmarks.  rt_profile_enable(ctx, 1) turns on stage
 * and round timing, (ctx, 2) round timing only (rt_profile_recon_rounds; two
 * events per run of round launches, no stage events), (ctx, 0) neither.
 * While stage timing is on, rt_segment_tile records HIP events on its own
 * stream at the boundaries of its stages:
 *   0 deconv       colour deconvolution (table, histogram, pixels)
 *   1 level_bound  frame connectivity of the upper level sets (CCL, 8 levels)
 *   2 recon        reconstruction rounds (one launch per round)
 *   3 fill_holes   FillHoles (background CCL)
 *   4 ccl          BWLabel with component area and bounding box
 *   5 objects      per-object Pre-Watershed + Watershed + relabel + area
 *   6 objects_big  the same for components larger than the LDS budget
 * Recording adds no synchronisation.  rt_profile_read synchronises the
 * recorded events, adds the elapsed milliseconds of each stage over all
 * calls since the last read into ms[i] and the number of kernel launches
 * into launches[i] (i < max_stages), clears the record and returns the number
 * of profiled calls.
 */
#define RT_PROF_STAGES 7
int rt_profile_enable(rt_ctx *ctx, int enable);
int rt_profile_read(rt_ctx *ctx, double *ms, int64_t *launches, int max_stages);
const char *rt_profile_stage_name(int stage);
/*
 * Timing of the reconstruction round kernel, recorded while profiling is
 * enabled (mode 1 or 2): a pair of HIP events on the call's stream around
 * each run of consecutive round launches (the launches between two host
 * checks of the worklist, or the one work-queue launch), so the time between
 * launches of a run counts as kernel time.  Returns the summed milliseconds,
 * the number of round launches and the number of 62 x 62 tile visits (tiles
 * processed, over all rounds) since the last read, synchronises the events
 * and clears the record.
 */
int rt_profile_recon_rounds(rt_ctx *ctx, double *kernel_ms, int64_t *launches, int64_t *tile_visits);
/*
 * Timing of the per-object kernels (profiling modes 1 and 2, outside graph
 * capture): cls 0 = small class (crops up to 32 x 32, and the components
 * erased by the first area threshold), 1 = medium (up to 64 x 64), 2 = large
 * LDS class.  kernel_ms = summed time between an event pair recorded around
 * each launch of the class on the stream it runs on; launches = launches
 * recorded; pixels = pixels of the components in the class's work list (the
 * sum of their areas, tallied on the device by a separate kernel after the
 * stage).  Reading synchronises and clears that class's figures.
 */
int rt_profile_objects(rt_ctx *ctx, int cls, double *kernel_ms, int64_t *launches, int64_t *pixels);

#ifdef __cplusplus
}
#endif
#endif
