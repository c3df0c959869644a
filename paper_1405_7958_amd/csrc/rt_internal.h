// Internal declarations shared by the host API and the HIP kernels of librtseg.
#pragma once
#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------------------
// context: device, scratch arena, pinned readback slot
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
    int recon_levels = 3;        // threshold levels of the connectivity lower bound
    int recon_round_batch = 8;   // propagation rounds launched between host checks
    int recon_max_sweeps = 64;   // in-tile sweeps before a tile re-queues itself
};

struct rt_ctx_impl {
    int device = 0;
    int n_cu = 256;
    Arena arena;
    int32_t *pinned = nullptr;   // small pinned host buffer for counter readback
    double *lut = nullptr;       // 3 x 256 FP64 deconvolution table (device)
    uint32_t stamp_epoch = 1;    // round stamps for the reconstruction worklists
    uint32_t *stamps = nullptr;  // per-tile stamp array (device)
    size_t stamps_cap = 0;
    Knobs knobs;
    // stage timing
    bool prof_on = false;
    std::vector<hipEvent_t> prof_events;   // (RT_PROF_STAGES + 1) per profiled call
    size_t prof_used = 0;                  // events in use
    int64_t prof_launches[RT_PROF_STAGES] = {};
    int prof_calls = 0;
};

int ensure_arena(rt_ctx_impl *c, size_t bytes);
int ensure_stamps(rt_ctx_impl *c, size_t ntiles);

// ---------------------------------------------------------------------------
// kernel launchers (all asynchronous on `s`)
// ---------------------------------------------------------------------------
struct StainParams {
    double rows[9];
    double scale;
};

// deconvolution
int launch_deconv_lut(const StainParams &sp, double *lut, int *status_dev, hipStream_t s);
int launch_deconv(const double *lut, double scale, const uint8_t *rgb, int64_t rgb_pitch, int w, int h,
                  float *ch, int64_t ch_pitch, uint8_t *hq, int64_t hq_pitch,
                  uint8_t *frame_init /*nullable: R0 = Hq on frame, 0 inside*/, int64_t fi_pitch,
                  uint32_t *hist /*nullable: 256 bins*/, int n_cu, hipStream_t s);

// connected components (union-find).  `ids` is a scratch int32 array of
// w*h + 1 entries: id 0 is a virtual node, pixel p has id p + 1.
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
    // outputs
    int32_t *labels; int64_t pitch_l;   // Labels: root id or 0
    uint8_t *fill; int64_t pitch_f;     // FillHoles: F0 | !frame-connected
    uint8_t *bound; int64_t pitch_r;    // LevelBound: bound = max(bound, level) where frame-connected
    uint8_t *bg_zero_mask; int64_t pitch_m;  // Labels: write 0 to this mask at background pixels (nullable)
    // per-component statistics (Labels, nullable): indexed by root id
    int32_t *st_area, *st_x0, *st_x1, *st_y0, *st_y1;
    int32_t *obj_list, *n_obj;     // roots registered here (nullable)
};
int launch_ccl(const CclArgs &a, hipStream_t s);

// reconstruction rounds
struct ReconArgs {
    int dtype;                     // RT_U8 / RT_I32
    int conn;
    int w, h;
    int64_t pitch;
    const void *mask;
    void *r;                       // in: initial values (already min(marker,mask)); out: result
    const uint8_t *domain;
};
int recon_init(int dtype, const void *marker, const void *mask, void *out, const uint8_t *domain, int w, int h,
               int64_t pitch, hipStream_t s);
int recon_rounds(rt_ctx_impl *c, const ReconArgs &a, hipStream_t s, int *rounds_out = nullptr);
int64_t recon_tiles(int w, int h);   // number of reconstruction tiles of a w x h image
int launch_select_levels(const uint32_t *hist, int n_levels, int32_t *levels, hipStream_t s);
int launch_frame_marker(const uint8_t *hq, int64_t pitch_hq, uint8_t *r, int64_t pitch_r, int w, int h,
                        hipStream_t s);

// area filter for labels produced by CCL (root ids)
int launch_area_filter(const int32_t *lab_in, int32_t *lab_out, uint8_t *mask_out, int w, int h, int64_t pitch,
                       int min_area, int max_area, int32_t *area_scratch, hipStream_t s);

// per-object watershed split (runs on the components registered by the CCL)
struct ObjArgs {
    int w, h;
    int64_t pitch;
    const int32_t *obj_list;
    const int32_t *n_obj;
    const int32_t *st_area, *st_x0, *st_x1, *st_y0, *st_y1;
    int32_t *labels;               // in: root id of each pixel's component; out: final labels
    uint8_t *mask;                 // out
    const uint8_t *seeds;          // nullable external seeds
    int h_seed;
    int min_area_pre;              // components below this area are erased
    int min_area, max_area;        // final area filter (max_area < 0: none)
    int32_t *n_kept;               // nullable: number of kept objects
    int32_t *list_m, *n_m;         // components deferred to the medium LDS class
    int32_t *big_list, *n_big;     // components deferred to the global-memory class
    void *big_scratch;             // global scratch slices for the global-memory class
    size_t big_scratch_bytes;
};
int launch_objects(const ObjArgs &a, int n_cu, hipStream_t s);
size_t big_object_bytes(int w, int h);

int launch_fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s);
int launch_count_zero(const uint8_t *m, int w, int h, int64_t pitch, int32_t *out, hipStream_t s);

}  // namespace rtseg
