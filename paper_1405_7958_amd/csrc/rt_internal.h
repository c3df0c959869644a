// Internal declarations shared by the host API and the HIP kernels of librtseg.
//
// Every stage kernel is batch-native: it receives a device array with one
// argument record per image and walks a combined space of work units (pixel
// chunks, 64 x 64 CCL tiles, 62 x 62 reconstruction tiles, components) with a
// persistent grid-stride loop.  A record's `unit0` is the first unit of its
// image; unit u belongs to the image i with unit0[i] <= u < unit0[i+1].  One
// tile is a batch of one.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rtseg.h"

namespace rtseg {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define RT_HIP(call)                                                        \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess) return ::rtseg::hip_fail(_e, #call);          \
    } while (0)

constexpr int MAX_BATCH = 64;   // images per launch (component codes carry a 6-bit image index)

// ---------------------------------------------------------------------------
// context: device, scratch arena, pinned staging
// ---------------------------------------------------------------------------
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    void reset() { off = 0; }
    // carve `bytes` (256-byte aligned); returns nullptr if the arena is too small
    void *take(size_t bytes) {
        size_t o = (off + 255) & ~size_t(255);
        if (o + bytes > cap) return nullptr;
        off = o + bytes;
        return base + o;
    }
};

struct Knobs {
    int recon_levels = 2;        // threshold levels of the connectivity lower bound
    int recon_level_mode = 1;    // 0: Hq quantiles 0.75..0.33; 1: band of consecutive values at recon_level_frac
    int recon_level_frac = 500;  // per mille of pixels with Hq >= the band's second-highest level
    int recon_round_batch = 8;   // propagation rounds launched between host checks
    int recon_max_sweeps = 64;   // in-tile sweeps before a tile re-queues itself
    int objects_path = 0;        // per-object class routing (ObjLists::path)
    int recon_mode = 0;          // 0: rounds with host checks; 1: one work-queue launch; 2: rounds, then the queue
    int recon_queue_after = 2;   // recon_mode 2: rounds launched before the work queue takes over
    int graph = 0;               // replay segmentation batches from captured HIP graphs
    int graph_rounds = 24;       // reconstruction rounds inside the first graph
    int recon_async = 0;         // 1: no host read of the worklist -- recon_async_rounds launched rounds,
                                 // then the device-side finish (segmentation entry points)
    int recon_async_rounds = 16;
    int objects_streams = 1;     // 1: the three per-object classes on three streams; 0: one after the other
};

// A captured segmentation batch: graph A = deconvolution, connectivity bound
// and the first `graph_rounds` reconstruction rounds; graph B = fill holes,
// labelling and the per-object stage.  `key` lists everything the launch
// parameters depend on.
struct GraphPair {
    std::vector<int64_t> key;
    hipGraphExec_t a = nullptr, b = nullptr;
    uint64_t last_use = 0;
};

constexpr int kStaging = 4;   // argument-record upload buffers per context

struct rt_ctx_impl {
    int device = 0;
    int n_cu = 256;
    Arena arena;
    int32_t *pinned = nullptr;   // small pinned host buffer for counter readback
    char *staging[kStaging] = {};       // pinned host staging for per-image argument records (a ring)
    size_t staging_cap = 0;             // bytes of each
    hipEvent_t staging_done[kStaging] = {};   // recorded after the last upload from each buffer
    bool staging_pending[kStaging] = {};
    int staging_next = 0;
    double *lut = nullptr;       // 3 x 256 FP64 deconvolution table (device)
    uint32_t *stamps = nullptr;  // per-tile stamp array (device)
    size_t stamps_cap = 0;
    Knobs knobs;
    hipStream_t cap_stream = nullptr;      // private stream for graph capture
    hipStream_t side_stream = nullptr;     // per-object classes beside the small class
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipStream_t side_stream2 = nullptr;    // the large LDS class beside the other two
    hipEvent_t join2_ev = nullptr;
    std::vector<GraphPair> graphs;         // small cache of captured batches
    uint64_t graph_clock = 0;
    int64_t graph_replays = 0, graph_captures = 0;
    int last_rounds = 0;
    int64_t recon_host_reads = 0;          // worklist counts the host has read (each a stream synchronisation)
    // stage timing
    bool prof_on = false;                  // round timing (modes 1 and 2)
    bool prof_stages = false;              // stage boundary events (mode 1)
    std::vector<hipEvent_t> prof_events;   // (RT_PROF_STAGES + 1) per profiled call
    size_t prof_used = 0;                  // events in use
    int64_t prof_launches[RT_PROF_STAGES] = {};
    int prof_calls = 0;
    std::vector<hipEvent_t> round_events;  // begin/end pairs around each run of consecutive round launches
    size_t round_used = 0;
    int64_t round_launches = 0;            // round launches inside those pairs
    unsigned long long *prof_visits = nullptr;   // device: tiles processed by the round kernel
    // per-object classes (small, medium, large LDS): begin/end event pairs
    // around each launch on the class's own stream, launches, and a device
    // counter per class of the pixels of the components in its list
    std::vector<hipEvent_t> obj_events[3];
    size_t obj_used[3] = {};
    int64_t obj_launches[3] = {};
    unsigned long long *prof_obj_px = nullptr;
    // host-resident tile streams: device slots (RGB in, mask, labels and count
    // out) and the upload / download streams with one event per slot and phase
    hipStream_t up_stream = nullptr, down_stream = nullptr;
    hipEvent_t slot_up[3] = {}, slot_comp[3] = {}, slot_down[3] = {};
    char *slots = nullptr;
    size_t slot_bytes = 0;
    // cross-tile stitching: per-tile outputs of one launch group
    char *stitch_buf = nullptr;
    size_t stitch_cap = 0;
};

int ensure_arena(rt_ctx_impl *c, size_t bytes);
int ensure_stamps(rt_ctx_impl *c, size_t ntiles);
int ensure_staging(rt_ctx_impl *c, size_t bytes);

// ---------------------------------------------------------------------------
// colour deconvolution
// ---------------------------------------------------------------------------
struct StainParams {
    double rows[9];
    double scale;
};
struct DeconvImg {
    const uint8_t *rgb;
    int64_t rgb_pitch;
    uint8_t *hq;
    int64_t hq_pitch;
    float *ch;                     // nullable
    int64_t ch_pitch;
    uint32_t *hist;                // nullable: HIST_COPIES x 256 bins (their sum is the histogram)
    int w, h;
    int64_t unit0;                 // first 4096-pixel chunk of this image
};
constexpr int DECONV_CHUNK = 4096;
constexpr int HIST_COPIES = 16;
int launch_deconv_lut(const StainParams &sp, double *lut, hipStream_t s);
int launch_deconv(const double *lut, double scale, const DeconvImg *imgs_dev, int n, int64_t total_units,
                  int n_cu, hipStream_t s);

// ---------------------------------------------------------------------------
// connected components (union-find).  `ids` is a scratch int32 array of
// w*h + 1 entries per level: id 0 is a virtual node, pixel p has id p + 1.
// ---------------------------------------------------------------------------
enum class CclPred { NonZero, Zero, TophatBg, Level };
enum class CclOut { Labels, FillHoles, LevelBound };
struct CclArgs {
    CclPred pred;
    CclOut out;
    int conn;
    bool frame_virtual;            // link frame pixels that satisfy the predicate to id 0
    int w, h;
    const uint8_t *a;              // NonZero/Zero: mask; TophatBg/Level: Hq
    const uint8_t *b;              // TophatBg: R
    int64_t pitch_a, pitch_b;
    int t;                         // TophatBg threshold
    const int32_t *levels;         // Level: device array of levels
    int n_levels;
    int32_t *ids;                  // w*h+1 (times n_levels for Level)
    int32_t *bt;                   // border table: ccl_border_ints(w, h) (times n_levels for Level)
    // outputs
    int32_t *labels; int64_t pitch_l;   // Labels: root id or 0
    uint8_t *fill; int64_t pitch_f;     // FillHoles: F0 | !frame-connected
    uint8_t *bound; int64_t pitch_r;    // LevelBound: bound = max(bound, level) where frame-connected
    uint8_t *zero_mask; int64_t pitch_m;     // Labels: this mask is cleared over the image (nullable; the per-object stage then writes every member pixel)
    // per-component statistics (Labels, nullable): indexed by root id
    int32_t *st_area, *st_x0, *st_x1, *st_y0, *st_y1;
    int32_t *obj_list, *n_obj;     // components registered here (nullable); entries are image << 25 | root
    int img;                       // index of this record in its batch
    int unit0;                     // first 64 x 64 tile of this image
};
int ccl_tiles(int w, int h);   // number of 64 x 64 CCL tiles of a w x h image
// ints of the CCL border table of a w x h image (256 per tile): for each
// border pixel of a tile, the id of its local root, or -1
inline size_t ccl_border_ints(int w, int h) { return (size_t)ccl_tiles(w, h) * 256; }
// All records of one launch share the predicate and output (and, in the
// multi-level mode, the number of levels).
int launch_ccl(const CclArgs *args_dev, int n, int total_units, int n_cu, hipStream_t s, CclPred pred, CclOut out,
               int n_levels = 1);

// ---------------------------------------------------------------------------
// reconstruction rounds
// ---------------------------------------------------------------------------
struct ReconImg {
    int w, h;
    int64_t pitch;
    const void *mask;
    void *r;                       // in: initial values (already min(marker,mask)); out: result
    const uint8_t *domain;         // nullable
    int ntx, nty;                  // reconstruction tiles per row / column
    int unit0;                     // first tile of this image in the batch
};
// dtype of the reconstruction calls for uint8 images with no domain (the
// fast round kernel); the API dtypes RT_U8 / RT_I32 select the general one
constexpr int RECON_U8_PLAIN = 101;
int64_t recon_tiles(int w, int h);   // number of 62 x 62 reconstruction tiles of a w x h image
int recon_init(int dtype, const void *marker, const void *mask, void *out, int w, int h, int64_t pitch,
               hipStream_t s);
// Worklists and counters of one reconstruction over `total` tiles (carved
// from the arena).
struct ReconRun {
    int32_t *lists = nullptr;      // two lists of `total` tile ids
    int32_t *cnt = nullptr;        // 3 rotating counters
    int total = 0;
    unsigned long long *ring = nullptr;   // work queue: 2*total entries
    unsigned int *qctl = nullptr;         // head, tail, pending, abort, finished
    unsigned int *inq = nullptr;          // per tile: queued
};
// bytes recon_prepare takes from the arena for `total` tiles
inline size_t recon_scratch_bytes(int total) {
    const size_t t = (size_t)(total > 0 ? total : 1);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al(sizeof(int32_t) * (2 * t + 4)) + al(8 * 2 * t) + al(32) + al(4 * t) + 1024;
}
int recon_prepare(rt_ctx_impl *c, int total, ReconRun &run);
// Enqueues rounds k0 .. k1-1 (no synchronisation; capturable).  All images
// share dtype and connectivity.
int recon_launch(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn, int k0,
                 int k1, hipStream_t s);
// Enqueues the device-side finish of rounds k0, k0 + 1, ... (one workgroup,
// no host read; capturable); k0 >= 1.
int recon_finish_device(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn,
                        int k0, hipStream_t s);
// Enqueues the work-queue propagation (one persistent launch; capturable).
// from_round > 0: seed the queue with the worklist round from_round - 1 left
// (rounds 0 .. from_round - 1 already enqueued on s); else with every tile
int recon_queue(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn,
                hipStream_t s, int from_round = 0);
// After recon_queue: whether a wave gave up waiting (synchronises `s`); the
// caller then finishes with recon_finish from round 0.
int recon_queue_aborted(rt_ctx_impl *c, const ReconRun &run, hipStream_t s, int *aborted);
// Reads the number of tiles queued for round k (synchronises `s`).
int recon_pending(rt_ctx_impl *c, const ReconRun &run, int k, hipStream_t s, int *pending);
// Runs rounds from k0 on until no tile is queued (synchronises `s` every
// `recon_round_batch` rounds).
int recon_finish(rt_ctx_impl *c, const ReconRun &run, const ReconImg *imgs_dev, int n, int dtype, int conn, int k0,
                 hipStream_t s, int *rounds_out = nullptr);
// recon_prepare + recon_finish from round 0; releases the worklists.
int recon_rounds(rt_ctx_impl *c, const ReconImg *imgs_dev, int n, int dtype, int conn, int total, hipStream_t s,
                 int *rounds_out = nullptr);

// Per-image bookkeeping of a segmentation batch.
struct BatchAux {
    uint32_t *hist;                // HIST_COPIES x 256 bins of Hq
    int32_t *levels;               // threshold levels of the connectivity bound
    int32_t *kept;                 // kept objects (device)
    int32_t *n_dev;                // nullable caller counter
    const uint8_t *hq;             // dense, pitch w
    uint8_t *R;                    // dense, pitch w
    int w, h;
    uint8_t *fg_out, *seeds_out;   // nullable caller maps (pitch out_pitch), zeroed at the start
    int64_t out_pitch;
};
int launch_batch_begin(const BatchAux *aux, int n, int32_t *shared_ctr, int n_ctr, hipStream_t s);
int launch_batch_levels(const BatchAux *aux, int n, int n_levels, int mode, int frac_permille, hipStream_t s);
int launch_batch_frame_marker(const BatchAux *aux, int n, hipStream_t s);
int launch_batch_end(const BatchAux *aux, int n, hipStream_t s);
int launch_batch_zero_maps(const BatchAux *aux, int n, hipStream_t s);

// area filter for labels produced by CCL (root ids)
int launch_area_filter(const int32_t *lab_in, int32_t *lab_out, uint8_t *mask_out, int w, int h, int64_t pitch,
                       int min_area, int max_area, int32_t *area_scratch, hipStream_t s);

// ---------------------------------------------------------------------------
// per-object watershed split (runs on the components registered by the CCL)
// ---------------------------------------------------------------------------
struct ObjArgs {                   // one record per image
    int w, h;
    int64_t pitch;
    const int32_t *st_area, *st_x0, *st_x1, *st_y0, *st_y1;
    int32_t *labels;               // in: root id of each pixel's component; out: final labels
    uint8_t *mask;                 // out
    const uint8_t *seeds;          // nullable external seeds
    int h_seed;
    int min_area_pre;              // components below this area are erased
    int min_area, max_area;        // final area filter (max_area < 0: none)
    int32_t *n_kept;               // nullable: number of kept objects of this image
    uint8_t *fg_out, *seeds_out;   // nullable (both or neither): foreground after the first
                                   // area threshold and its seeds; zeroed by the caller
};
struct ObjLists {                  // shared by the batch; entries are image << 25 | root
    const int32_t *obj, *n_obj;
    int32_t *list_s, *n_s;         // small class
    int32_t *list_m, *n_m;         // deferred to the medium LDS class
    int32_t *list_l, *n_l;         // deferred to the large LDS class
    int32_t *big, *n_big;          // deferred to the global-memory classes
    int32_t *huge, *n_huge;        // crops above MID_MAX_PX pixels
    void *mid_scratch;             // many slices for crops up to MID_MAX_PX pixels
    size_t mid_slice_bytes;
    int mid_slices;
    void *big_scratch;             // a few slices for the largest crop of the batch
    size_t big_slice_bytes;
    int big_slices;
    int path = 0;                  // 0: small / medium register classes, then large LDS;
                                   // 1: small register class, then large LDS;
                                   // 2: large LDS class for every crop that fits
    int32_t *list_e = nullptr, *n_e = nullptr;     // components below the first area threshold, to erase
    int32_t *list_sd = nullptr, *n_sd = nullptr;   // small components with several seeds (or any, with
                                   // external seeds or seed maps wanted), deferred by the first small-class
                                   // pass to the full one; n_sd zeroed by the caller
};
constexpr int64_t MID_MAX_PX = 257 * 256;   // crops up to 256 x 256
// Optional side stream for the small class, joined back into the caller's
// stream with the two events before the global-memory classes.
struct ObjStreams {
    hipStream_t side, side2;
    hipEvent_t fork, join, join2;
    hipEvent_t timing[3][2] = {};  // nullable: begin/end of the small, medium and large class launches
};
// `before_big` (nullable) is recorded on `s` at the end of the LDS classes.
int launch_objects(const ObjArgs *args_dev, const ObjLists &lists, int n_cu, hipStream_t s,
                   hipEvent_t before_big = nullptr, const ObjStreams *par = nullptr);
// profiling: out[k] += pixels of the components in LDS class k's list (after the stage)
int launch_objects_tally(const ObjArgs *args_dev, const ObjLists &lists, unsigned long long *out, int n_cu,
                         hipStream_t s);
size_t big_object_bytes(int w, int h);   // one slice for the largest crop of a w x h image
size_t mid_object_bytes(int w, int h);   // one slice for a crop of at most MID_MAX_PX pixels
// number of mid slices for a launch group of `pixels` pixels
inline int mid_slices_for(int64_t pixels) {
    return (int)std::max<int64_t>(8, std::min<int64_t>(128, pixels / 65536));
}

// ---------------------------------------------------------------------------
// feature computation (per nucleus)
// ---------------------------------------------------------------------------
struct NucAcc {                    // step-1 intermediates of one nucleus
    int64_t area, perim, sx, sy, sxx, syy, sxy, gsum, gsum2, gmax;   // sums relative to the root pixel
    uint32_t hist[256];
    uint32_t glcm[RT_FEAT_GLCM_LEVELS * RT_FEAT_GLCM_LEVELS];
    uint32_t ghist[RT_FEAT_GRAD_BINS];
};
struct FeatArgs {
    const int32_t *labels;
    int64_t lab_pitch;
    const uint8_t *hq;
    int64_t hq_pitch;
    int w, h;
    int max_nuclei;
    int32_t *row_off;              // h + 1: root counts, then row offsets; [h] = total
    int32_t *map;                  // w*h: label - 1 -> rank (written at roots only)
    int32_t *box;                  // 4 per nucleus: x0, y0, x1, y1
    NucAcc *acc;                   // per nucleus
    int32_t *labels_out;           // max_nuclei
    double *feats;                 // max_nuclei x RT_NFEAT
    int64_t *counts;               // nullable: max_nuclei x RT_FEAT_NCOUNT
    int32_t *n_out;                // nullable: number of nuclei
};
int launch_features(const FeatArgs &a, int n_cu, hipStream_t s);

// ---------------------------------------------------------------------------
// pre-processing: flat-disk erosion / dilation, ReconToNuclei markers, RBC maps
// ---------------------------------------------------------------------------
struct MorphArgs {
    const uint8_t *in;
    int64_t in_pitch;
    uint8_t *out;
    int64_t out_pitch;
    int w, h, radius;
    int span[2 * RT_MORPH_MAX_RADIUS + 1];   // half-width of the disk at row offset dy (index dy + radius)
};
int launch_morph(const MorphArgs &a, bool erode, int n_cu, hipStream_t s);
int launch_frame_marker(const uint8_t *hq, int64_t hq_pitch, uint8_t *r, int64_t r_pitch, int w, int h,
                        hipStream_t s);
int launch_tophat(const uint8_t *hq, int64_t hq_pitch, const uint8_t *r, int64_t r_pitch, uint8_t *f0,
                  int64_t f0_pitch, int w, int h, int t, hipStream_t s);
int launch_rbc_maps(const uint8_t *rgb, int64_t rgb_pitch, int w, int h, int t_strong, int t_weak, uint8_t *marker,
                    uint8_t *mask, int64_t pitch, hipStream_t s);

// ---------------------------------------------------------------------------
// cross-tile stitching
// ---------------------------------------------------------------------------
struct StitchTile {
    const int32_t *labels;         // the extended tile's labels (dense, pitch ew)
    const uint8_t *hq;             // its Hq (dense, pitch ew), read when hq_out is set
    int ex0, ey0, ew, eh;          // extended region in slide coordinates
    int x0, y0, x1, y1;            // core [x0, x1) x [y0, y1)
};
struct StitchGroup {               // passed by value: at most MAX_BATCH tiles
    StitchTile t[MAX_BATCH];
    int n;
    int W;
    int32_t *labels;               // slide labels, pitch out_pitch (INT32_MAX = not yet written)
    uint8_t *hq_out;               // nullable slide Hq
    int64_t out_pitch;
    int32_t *n_objects;            // nullable
};
int launch_stitch_init(int32_t *labels, int64_t pitch, int W, int H, int32_t *n_objects, int n_cu, hipStream_t s);
int launch_stitch(const StitchGroup &g, int n_cu, hipStream_t s);
int launch_stitch_final(int32_t *labels, uint8_t *mask, int64_t pitch, int W, int H, int n_cu, hipStream_t s);

int launch_fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s);

// Most components a w x h image can hold.  8-connectivity: two pixels of one
// 2 x 2 block are always adjacent, so each block meets at most one component.
// 4-connectivity: the same holds for each horizontal pair of a row (a
// checkerboard reaches ceil(w/2) per row).
inline size_t max_components(int w, int h, int conn) {
    return conn == 4 ? (((size_t)w + 1) / 2) * (size_t)h : ((size_t)w / 2 + 1) * ((size_t)h / 2 + 1);
}

// BWLabel on the fixed device array of noalloc.hip (no allocation).  The
// array's device address is looked up by noalloc_init_device, once per
// device, with that device current.
int noalloc_init_device(int device);
size_t noalloc_ccl_bytes(int w, int h, int conn, bool want_count);
int ccl_noalloc(int device, int n_cu, const uint8_t *mask, int32_t *labels, int w, int h, int64_t pitch, int conn,
                int32_t *n_out_dev, hipStream_t s);
// zeroes a pitched w x h uint8 image
int launch_zero_u8(uint8_t *p, int64_t pitch, int w, int h, hipStream_t s);
// Surrogate maps: fg = [p_fg >= 0.5], seeds = [p_seed >= 0.5]; counts[0] +=
// pixels with p_fg >= 0.25, counts[1] += pixels with 0.25 <= p_fg < 0.75,
// counts[2], counts[3] the same for p_seed.
int launch_surrogate_maps(const float *p_fg, const float *p_seed, int w, int h, uint8_t *fg, uint8_t *seeds,
                          int32_t *counts, hipStream_t s);

}  // namespace rtseg
