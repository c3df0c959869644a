// Host side of the C ABI: argument checks, scratch management and the launch
// sequence of every entry point.  All arithmetic runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "rt_internal.h"

struct rt_ctx : rtseg::rt_ctx_impl {};

namespace rtseg {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
    if (e == hipSuccess) return RT_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return RT_EDEVICE;
}

int ensure_arena(rt_ctx_impl *c, size_t bytes) {
    c->arena.reset();
    if (bytes <= c->arena.cap) return RT_OK;
    if (c->arena.base) {
        RT_HIP(hipDeviceSynchronize());
        RT_HIP(hipFree(c->arena.base));
        c->arena.base = nullptr;
        c->arena.cap = 0;
    }
    size_t cap = (bytes + (size_t(1) << 20)) & ~((size_t(1) << 20) - 1);
    void *p = nullptr;
    if (hipMalloc(&p, cap) != hipSuccess) {
        (void)hipGetLastError();
        set_error("scratch allocation of %zu bytes failed", cap);
        return RT_ENOMEM;
    }
    c->arena.base = (char *)p;
    c->arena.cap = cap;
    return RT_OK;
}

int ensure_stamps(rt_ctx_impl *c, size_t ntiles) {
    if (ntiles <= c->stamps_cap) return RT_OK;
    if (c->stamps) {
        RT_HIP(hipDeviceSynchronize());
        RT_HIP(hipFree(c->stamps));
    }
    size_t cap = std::max<size_t>(ntiles, 4096);
    if (hipMalloc(&c->stamps, cap * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        c->stamps = nullptr;
        c->stamps_cap = 0;
        set_error("stamp allocation failed");
        return RT_ENOMEM;
    }
    RT_HIP(hipMemset(c->stamps, 0, cap * sizeof(uint32_t)));
    c->stamps_cap = cap;
    c->stamp_epoch = 1;
    return RT_OK;
}

}  // namespace rtseg

using namespace rtseg;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool bad_size(int32_t w, int32_t h) { return w <= 0 || h <= 0 || (int64_t)w * h >= (int64_t(1) << 31) - 1; }

#define CHECK(cond, ...)                 \
    do {                                 \
        if (!(cond)) {                   \
            set_error(__VA_ARGS__);      \
            return RT_EINVAL;            \
        }                                \
    } while (0)

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// host-side validity check of the stain matrix (argument validation only;
// the table itself is built on the device)
bool stain_ok(const double r[9]) {
    double M[3][3];
    for (int i = 0; i < 3; ++i) {
        double n = std::sqrt(r[3 * i] * r[3 * i] + r[3 * i + 1] * r[3 * i + 1] + r[3 * i + 2] * r[3 * i + 2]);
        if (i < 2 && !(n > 0.0)) return false;
        for (int k = 0; k < 3; ++k) M[i][k] = n > 0.0 ? r[3 * i + k] / n : 0.0;
    }
    if (M[2][0] == 0.0 && M[2][1] == 0.0 && M[2][2] == 0.0) {
        double c0 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
        double c1 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
        double c2 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        double n = std::sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        if (!(n > 1e-12)) return false;
        M[2][0] = c0 / n;
        M[2][1] = c1 / n;
        M[2][2] = c2 / n;
    }
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                 M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                 M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    return std::fabs(det) > 1e-12;
}

int set_dev(rt_ctx *c) { return hip_fail(hipSetDevice(c->device), "hipSetDevice"); }

const char *kStageNames[RT_PROF_STAGES] = {"deconv", "level_bound", "recon", "fill_holes", "ccl", "objects",
                                           "objects_big"};

// Records the boundary event `k` (0..RT_PROF_STAGES) of the current profiled call.
int prof_mark(rt_ctx *c, int k, hipStream_t s) {
    if (!c->prof_on) return RT_OK;
    size_t idx = c->prof_used + (size_t)k;
    while (c->prof_events.size() <= idx) {
        hipEvent_t ev;
        RT_HIP(hipEventCreate(&ev));
        c->prof_events.push_back(ev);
    }
    RT_HIP(hipEventRecord(c->prof_events[idx], s));
    if (k == RT_PROF_STAGES) {
        c->prof_used += RT_PROF_STAGES + 1;
        c->prof_calls++;
    }
    return RT_OK;
}

// Scratch layout of one CCL: ids (w*h+1) per level.
size_t ccl_ids_bytes(int w, int h, int nlev) { return al(sizeof(int32_t) * ((size_t)w * h + 1) * nlev); }

struct CompScratch {
    int32_t *ids, *area, *x0, *x1, *y0, *y1, *obj, *list_m, *big;
    int32_t *n_obj, *n_m, *n_big, *n_kept;
    void *big_scratch;
    size_t big_bytes;
    size_t max_obj;
};

// Scratch of BWLabel + the per-object stage: component ids, statistics and
// lists, plus slices for crops too large for LDS (4 slices of the largest
// possible crop).
size_t comp_scratch_bytes(int w, int h) {
    size_t n1 = (size_t)w * h + 1;
    size_t max_obj = ((size_t)w / 2 + 1) * ((size_t)h / 2 + 1);
    return ccl_ids_bytes(w, h, 1) + 5 * al(sizeof(int32_t) * n1) + 3 * al(sizeof(int32_t) * max_obj) +
           al(sizeof(int32_t) * 8) + 4 * al(big_object_bytes(w, h));
}

int carve_comp(rt_ctx *c, int w, int h, CompScratch &cs) {
    size_t n1 = (size_t)w * h + 1;
    cs.max_obj = ((size_t)w / 2 + 1) * ((size_t)h / 2 + 1);
    cs.ids = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.area = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.x0 = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.x1 = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.y0 = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.y1 = (int32_t *)c->arena.take(sizeof(int32_t) * n1);
    cs.obj = (int32_t *)c->arena.take(sizeof(int32_t) * cs.max_obj);
    cs.list_m = (int32_t *)c->arena.take(sizeof(int32_t) * cs.max_obj);
    cs.big = (int32_t *)c->arena.take(sizeof(int32_t) * cs.max_obj);
    int32_t *ctr = (int32_t *)c->arena.take(sizeof(int32_t) * 8);
    cs.big_bytes = 4 * al(big_object_bytes(w, h));
    cs.big_scratch = c->arena.take(cs.big_bytes);
    if (!cs.ids || !cs.area || !cs.x0 || !cs.x1 || !cs.y0 || !cs.y1 || !cs.obj || !cs.list_m || !cs.big || !ctr ||
        !cs.big_scratch) {
        set_error("scratch arena too small");
        return RT_ENOMEM;
    }
    cs.n_obj = ctr;
    cs.n_m = ctr + 1;
    cs.n_big = ctr + 2;
    cs.n_kept = ctr + 3;
    return RT_OK;
}

// BWLabel (8-connected) with statistics, then the per-object watershed.
int components_and_watershed(rt_ctx *c, const uint8_t *fg, int64_t pitch_fg, const uint8_t *seeds, int h_seed,
                             int min_area_pre, int min_area, int max_area, int32_t *labels, uint8_t *mask,
                             int64_t pitch, int w, int h, CompScratch &cs, int32_t *n_kept_out, hipStream_t s) {
    int e = launch_fill_i32(cs.n_obj, 0, 4, s);
    if (e) return e;
    CclArgs A{};
    A.pred = CclPred::NonZero;
    A.out = CclOut::Labels;
    A.conn = 8;
    A.frame_virtual = false;
    A.w = w;
    A.h = h;
    A.a = fg;
    A.pitch_a = pitch_fg;
    A.ids = cs.ids;
    A.labels = labels;
    A.pitch_l = pitch;
    A.bg_zero_mask = mask;
    A.pitch_m = pitch;
    A.st_area = cs.area;
    A.st_x0 = cs.x0;
    A.st_x1 = cs.x1;
    A.st_y0 = cs.y0;
    A.st_y1 = cs.y1;
    A.obj_list = cs.obj;
    A.n_obj = cs.n_obj;
    e = launch_ccl(A, s);
    if (e) return e;
    e = prof_mark(c, 5, s);
    if (e) return e;
    c->prof_launches[4] += 4;
    ObjArgs o{};
    o.w = w;
    o.h = h;
    o.pitch = pitch;
    o.obj_list = cs.obj;
    o.n_obj = cs.n_obj;
    o.st_area = cs.area;
    o.st_x0 = cs.x0;
    o.st_x1 = cs.x1;
    o.st_y0 = cs.y0;
    o.st_y1 = cs.y1;
    o.labels = labels;
    o.mask = mask;
    o.seeds = seeds;
    o.h_seed = h_seed;
    o.min_area_pre = min_area_pre;
    o.min_area = min_area;
    o.max_area = max_area;
    o.n_kept = cs.n_kept;
    o.list_m = cs.list_m;
    o.n_m = cs.n_m;
    o.big_list = cs.big;
    o.n_big = cs.n_big;
    o.big_scratch = cs.big_scratch;
    o.big_scratch_bytes = cs.big_bytes;
    e = launch_objects(o, c->n_cu, s);
    if (e) return e;
    e = prof_mark(c, 6, s);
    if (e) return e;
    c->prof_launches[5] += 3;
    e = prof_mark(c, 7, s);
    if (e) return e;
    if (n_kept_out) RT_HIP(hipMemcpyAsync(n_kept_out, cs.n_kept, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    return RT_OK;
}

}  // namespace

extern "C" {

const char *rt_last_error(void) { return g_err; }

void rt_seg_params_default(rt_seg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->size = sizeof(rt_seg_params);
    const double st[9] = {0.650, 0.704, 0.286, 0.072, 0.990, 0.105, 0.0, 0.0, 0.0};
    std::memcpy(p->stain_rows, st, sizeof st);
    p->hq_scale = 85.0;
    p->t_fg = 16;
    p->min_area = 20;
    p->max_area = 1000;
    p->h_seed = 3;
    p->conn = 8;
}

int rt_ctx_create(int device, rt_ctx **out) {
    CHECK(out != nullptr, "rt_ctx_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    RT_HIP(hipGetDeviceCount(&ndev));
    CHECK(device >= 0 && device < ndev, "rt_ctx_create: device %d out of range (%d devices)", device, ndev);
    RT_HIP(hipSetDevice(device));
    rt_ctx *c = new rt_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    if (hipHostMalloc((void **)&c->pinned, 4096, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&c->lut, 768 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        if (c->pinned) (void)hipHostFree(c->pinned);
        delete c;
        set_error("rt_ctx_create: allocation failed");
        return RT_ENOMEM;
    }
    *out = c;
    return RT_OK;
}

int rt_ctx_destroy(rt_ctx *c) {
    if (!c) return RT_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->arena.base) (void)hipFree(c->arena.base);
    if (c->stamps) (void)hipFree(c->stamps);
    if (c->lut) (void)hipFree(c->lut);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t ev : c->prof_events) (void)hipEventDestroy(ev);
    delete c;
    return RT_OK;
}

int rt_sync(rt_ctx *c, void *stream) {
    CHECK(c, "rt_sync: ctx is NULL");
    int e = set_dev(c);
    if (e) return e;
    RT_HIP(hipStreamSynchronize(as_stream(stream)));
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int rt_deconv(rt_ctx *c, const uint8_t *rgb, int64_t rgb_pitch, int32_t w, int32_t h, const double stain[9],
              double scale, float *ch, int64_t ch_pitch, uint8_t *hq, int64_t hq_pitch, void *stream) {
    CHECK(c && rgb && stain && hq, "rt_deconv: null argument");
    CHECK(!bad_size(w, h), "rt_deconv: bad size %dx%d", w, h);
    CHECK(rgb_pitch >= 3LL * w && hq_pitch >= w && (!ch || ch_pitch >= w), "rt_deconv: pitch smaller than width");
    CHECK(stain_ok(stain), "rt_deconv: singular stain matrix");
    CHECK(std::isfinite(scale), "rt_deconv: bad scale");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    StainParams sp;
    std::memcpy(sp.rows, stain, sizeof sp.rows);
    sp.scale = scale;
    e = launch_deconv_lut(sp, c->lut, nullptr, s);
    if (e) return e;
    return launch_deconv(c->lut, scale, rgb, rgb_pitch, w, h, ch, ch_pitch, hq, hq_pitch, nullptr, 0, nullptr,
                         c->n_cu, s);
}

int rt_morph_recon(rt_ctx *c, int dtype, const void *marker, const void *mask, void *out, const uint8_t *domain,
                   int32_t w, int32_t h, int64_t pitch, int conn, void *stream) {
    CHECK(c && marker && mask && out, "rt_morph_recon: null argument");
    CHECK(dtype == RT_U8 || dtype == RT_I32, "rt_morph_recon: bad dtype %d", dtype);
    CHECK(conn == 4 || conn == 8, "rt_morph_recon: conn must be 4 or 8");
    CHECK(!bad_size(w, h) && pitch >= w, "rt_morph_recon: bad size");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    int64_t ntiles = recon_tiles(w, h);
    e = ensure_arena(c, al(sizeof(int32_t) * (2 * ntiles + 4)) + 4096);
    if (e) return e;
    e = recon_init(dtype, marker, mask, out, domain, w, h, pitch, s);
    if (e) return e;
    ReconArgs ra{dtype, conn, w, h, pitch, mask, out, domain};
    return recon_rounds(c, ra, s);
}

int rt_fill_holes(rt_ctx *c, const uint8_t *in, uint8_t *out, int32_t w, int32_t h, int64_t pitch, int bg_conn,
                  void *stream) {
    CHECK(c && in && out, "rt_fill_holes: null argument");
    CHECK(bg_conn == 4 || bg_conn == 8, "rt_fill_holes: bg_conn must be 4 or 8");
    CHECK(!bad_size(w, h) && pitch >= w, "rt_fill_holes: bad size");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    e = ensure_arena(c, ccl_ids_bytes(w, h, 1) + 4096);
    if (e) return e;
    CclArgs A{};
    A.pred = CclPred::Zero;
    A.out = CclOut::FillHoles;
    A.conn = bg_conn;
    A.frame_virtual = true;
    A.w = w;
    A.h = h;
    A.a = in;
    A.pitch_a = pitch;
    A.ids = (int32_t *)c->arena.take(sizeof(int32_t) * ((size_t)w * h + 1));
    A.fill = out;
    A.pitch_f = pitch;
    return launch_ccl(A, s);
}

int rt_ccl(rt_ctx *c, const uint8_t *mask, int32_t *labels, int32_t w, int32_t h, int64_t pitch, int conn,
           int32_t *n_out_dev, void *stream) {
    CHECK(c && mask && labels, "rt_ccl: null argument");
    CHECK(conn == 4 || conn == 8, "rt_ccl: conn must be 4 or 8");
    CHECK(!bad_size(w, h) && pitch >= w, "rt_ccl: bad size");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    size_t max_obj = ((size_t)w / 2 + 1) * ((size_t)h / 2 + 1);
    e = ensure_arena(c, ccl_ids_bytes(w, h, 1) + al(sizeof(int32_t) * max_obj) + al(64) + 4096);
    if (e) return e;
    CclArgs A{};
    A.pred = CclPred::NonZero;
    A.out = CclOut::Labels;
    A.conn = conn;
    A.w = w;
    A.h = h;
    A.a = mask;
    A.pitch_a = pitch;
    A.ids = (int32_t *)c->arena.take(sizeof(int32_t) * ((size_t)w * h + 1));
    A.labels = labels;
    A.pitch_l = pitch;
    if (n_out_dev) {
        A.obj_list = (int32_t *)c->arena.take(sizeof(int32_t) * max_obj);
        A.n_obj = n_out_dev;
        e = launch_fill_i32(n_out_dev, 0, 1, s);
        if (e) return e;
    }
    return launch_ccl(A, s);
}

int rt_area_filter(rt_ctx *c, const int32_t *lab_in, int32_t *lab_out, uint8_t *mask_out, int32_t w, int32_t h,
                   int64_t pitch, int32_t min_area, int32_t max_area, void *stream) {
    CHECK(c && lab_in && lab_out, "rt_area_filter: null argument");
    CHECK(!bad_size(w, h) && pitch >= w, "rt_area_filter: bad size");
    CHECK(min_area <= max_area, "rt_area_filter: min_area > max_area");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    e = ensure_arena(c, al(sizeof(int32_t) * ((size_t)w * h + 1)) + 4096);
    if (e) return e;
    int32_t *area = (int32_t *)c->arena.take(sizeof(int32_t) * ((size_t)w * h + 1));
    return launch_area_filter(lab_in, lab_out, mask_out, w, h, pitch, min_area, max_area, area, s);
}

int rt_watershed(rt_ctx *c, const uint8_t *fg, const uint8_t *seeds, int32_t h_seed, int32_t *labels_out,
                 uint8_t *mask_out, int32_t w, int32_t h, int64_t pitch, void *stream) {
    CHECK(c && fg && labels_out && mask_out, "rt_watershed: null argument");
    CHECK(!bad_size(w, h) && pitch >= w, "rt_watershed: bad size");
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    e = ensure_arena(c, comp_scratch_bytes(w, h) + 8192);
    if (e) return e;
    CompScratch cs;
    e = carve_comp(c, w, h, cs);
    if (e) return e;
    const bool prof = c->prof_on;
    c->prof_on = false;  // stage events belong to rt_segment_tile
    e = components_and_watershed(c, fg, pitch, seeds, h_seed, 0, 0, -1, labels_out, mask_out, pitch, w, h, cs,
                                 nullptr, s);
    c->prof_on = prof;
    return e;
}

int rt_segment_tile(rt_ctx *c, const uint8_t *rgb, int64_t rgb_pitch, int32_t w, int32_t h,
                    const rt_seg_params *p, uint8_t *mask_out, int32_t *labels_out, int64_t out_pitch,
                    int32_t *n_objects_dev, uint8_t *hq_out, void *stream) {
    CHECK(c && rgb && p && mask_out && labels_out, "rt_segment_tile: null argument");
    CHECK(p->size == sizeof(rt_seg_params), "rt_segment_tile: params.size mismatch");
    CHECK(!bad_size(w, h), "rt_segment_tile: bad size %dx%d", w, h);
    CHECK(rgb_pitch >= 3LL * w && out_pitch >= w, "rt_segment_tile: pitch smaller than width");
    CHECK(p->conn == 8, "rt_segment_tile: foreground connectivity must be 8");
    CHECK(p->min_area <= p->max_area, "rt_segment_tile: min_area > max_area");
    CHECK(stain_ok(p->stain_rows), "rt_segment_tile: singular stain matrix");
    if (hq_out && out_pitch != w) {
        set_error("rt_segment_tile: hq_out needs out_pitch == w");
        return RT_EUNSUPPORTED;
    }
    int e = set_dev(c);
    if (e) return e;
    hipStream_t s = as_stream(stream);
    const size_t N = (size_t)w * h;
    const int nlev = c->knobs.recon_levels;
    const int64_t ntiles = recon_tiles(w, h);
    size_t need = 3 * al(N) + al(256 * 4) + al(64) +
                  std::max(ccl_ids_bytes(w, h, std::max(nlev, 1)) + al(sizeof(int32_t) * (2 * ntiles + 4)),
                           comp_scratch_bytes(w, h)) + 16384;
    e = ensure_arena(c, need);
    if (e) return e;
    uint8_t *hq = hq_out ? hq_out : (uint8_t *)c->arena.take(N);
    const int64_t hq_pitch = hq_out ? out_pitch : w;
    uint8_t *R = (uint8_t *)c->arena.take(N);
    uint8_t *F = (uint8_t *)c->arena.take(N);
    uint32_t *hist = (uint32_t *)c->arena.take(256 * 4);
    int32_t *levels = (int32_t *)c->arena.take(64);
    const size_t mark = c->arena.off;  // the later CCL scratch reuses the level ids
    int32_t *lev_ids = (int32_t *)c->arena.take(sizeof(int32_t) * (N + 1) * std::max(nlev, 1));
    if (!hq || !R || !F || !hist || !levels || !lev_ids) {
        set_error("rt_segment_tile: scratch arena too small");
        return RT_ENOMEM;
    }
    // only rt_segment_tile records stage events
    const bool prof = c->prof_on;
    struct ProfGuard {
        rt_ctx *c;
        bool on;
        ~ProfGuard() { c->prof_on = on; }
    } guard{c, prof};
    e = prof_mark(c, 0, s);
    if (e) return e;
    // 1. colour deconvolution + histogram of Hq
    StainParams sp;
    std::memcpy(sp.rows, p->stain_rows, sizeof sp.rows);
    sp.scale = p->hq_scale;
    e = launch_deconv_lut(sp, c->lut, nullptr, s);
    if (e) return e;
    e = launch_fill_i32((int32_t *)hist, 0, 256, s);
    if (e) return e;
    e = launch_deconv(c->lut, p->hq_scale, rgb, rgb_pitch, w, h, nullptr, 0, hq, hq_pitch, nullptr, 0, hist,
                      c->n_cu, s);
    if (e) return e;
    e = prof_mark(c, 1, s);
    if (e) return e;
    c->prof_launches[0] += 3;
    // 2. ReconToNuclei: start from the frame marker raised by the frame
    //    connectivity of a few upper level sets, then propagate
    if (nlev > 0) {
        e = launch_select_levels(hist, nlev, levels, s);
        if (e) return e;
        CclArgs A{};
        A.pred = CclPred::Level;
        A.out = CclOut::LevelBound;
        A.conn = 8;
        A.frame_virtual = true;
        A.w = w;
        A.h = h;
        A.a = hq;
        A.pitch_a = hq_pitch;
        A.levels = levels;
        A.n_levels = nlev;
        A.ids = lev_ids;
        A.bound = R;
        A.pitch_r = w;
        e = launch_ccl(A, s);
        if (e) return e;
        c->prof_launches[1] += 4 + nlev;
    } else {
        e = launch_frame_marker(hq, hq_pitch, R, w, w, h, s);
        if (e) return e;
        c->prof_launches[1] += 1;
    }
    e = prof_mark(c, 2, s);
    if (e) return e;
    {
        ReconArgs ra{RT_U8, 8, w, h, (int64_t)w, hq, R, nullptr};
        int rounds = 0;
        e = recon_rounds(c, ra, s, &rounds);
        if (e) return e;
        e = prof_mark(c, 3, s);
        if (e) return e;
        c->prof_launches[2] += rounds;
    }
    // 3. F0 = [Hq - R >= t]; FillHoles through the 4-connected background
    {
        c->arena.off = mark;
        int32_t *ids = (int32_t *)c->arena.take(sizeof(int32_t) * (N + 1));
        CclArgs A{};
        A.pred = CclPred::TophatBg;
        A.out = CclOut::FillHoles;
        A.conn = 4;
        A.frame_virtual = true;
        A.w = w;
        A.h = h;
        A.a = hq;
        A.b = R;
        A.pitch_a = hq_pitch;
        A.pitch_b = w;
        A.t = p->t_fg;
        A.ids = ids;
        A.fill = F;
        A.pitch_f = w;
        e = launch_ccl(A, s);
        if (e) return e;
        e = prof_mark(c, 4, s);
        if (e) return e;
        c->prof_launches[3] += 4;
    }
    // 4-8. BWLabel + AreaThreshold + Pre-Watershed/Watershed + relabel + AreaThreshold
    c->arena.off = mark;
    CompScratch cs;
    e = carve_comp(c, w, h, cs);
    if (e) return e;
    return components_and_watershed(c, F, w, nullptr, p->h_seed, p->min_area, p->min_area, p->max_area, labels_out,
                                    mask_out, out_pitch, w, h, cs, n_objects_dev, s);
}

int rt_set_knob(rt_ctx *c, const char *name, int value) {
    CHECK(c && name, "rt_set_knob: null argument");
    std::string n(name);
    if (n == "recon_levels") {
        CHECK(value >= 0 && value <= 8, "rt_set_knob: recon_levels must be 0..8");
        c->knobs.recon_levels = value;
    } else if (n == "recon_round_batch") {
        CHECK(value >= 1 && value <= 64, "rt_set_knob: recon_round_batch must be 1..64");
        c->knobs.recon_round_batch = value;
    } else if (n == "recon_max_sweeps") {
        CHECK(value >= 1 && value <= 1024, "rt_set_knob: recon_max_sweeps must be 1..1024");
        c->knobs.recon_max_sweeps = value;
    } else {
        set_error("rt_set_knob: unknown knob '%s'", name);
        return RT_EINVAL;
    }
    return RT_OK;
}

int rt_get_knob(rt_ctx *c, const char *name, int *value) {
    CHECK(c && name && value, "rt_get_knob: null argument");
    std::string n(name);
    if (n == "recon_levels")
        *value = c->knobs.recon_levels;
    else if (n == "recon_round_batch")
        *value = c->knobs.recon_round_batch;
    else if (n == "recon_max_sweeps")
        *value = c->knobs.recon_max_sweeps;
    else {
        set_error("rt_get_knob: unknown knob '%s'", name);
        return RT_EINVAL;
    }
    return RT_OK;
}

int rt_profile_enable(rt_ctx *c, int enable) {
    CHECK(c, "rt_profile_enable: ctx is NULL");
    c->prof_on = enable != 0;
    return RT_OK;
}

const char *rt_profile_stage_name(int stage) {
    return (stage >= 0 && stage < RT_PROF_STAGES) ? kStageNames[stage] : "";
}

int rt_profile_read(rt_ctx *c, double *ms, int64_t *launches, int max_stages) {
    CHECK(c && ms && launches, "rt_profile_read: null argument");
    int e = set_dev(c);
    if (e) return e;
    const int ns = std::min(max_stages, (int)RT_PROF_STAGES);
    for (int i = 0; i < ns; ++i) {
        ms[i] = 0.0;
        launches[i] = c->prof_launches[i];
    }
    const size_t per = RT_PROF_STAGES + 1;
    for (size_t b = 0; b + per <= c->prof_used; b += per) {
        RT_HIP(hipEventSynchronize(c->prof_events[b + per - 1]));
        for (int i = 0; i < ns; ++i) {
            float t = 0.f;
            RT_HIP(hipEventElapsedTime(&t, c->prof_events[b + i], c->prof_events[b + i + 1]));
            ms[i] += t;
        }
    }
    int calls = c->prof_calls;
    c->prof_used = 0;
    c->prof_calls = 0;
    for (int i = 0; i < RT_PROF_STAGES; ++i) c->prof_launches[i] = 0;
    return calls;
}

}  // extern "C"
