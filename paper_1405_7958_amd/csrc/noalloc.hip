// rt_ccl_noalloc: BWLabel with its scratch in a fixed device array, for
// callers that cannot allocate device or pinned host memory during a call.
//
// The array `scratch` lives in this code object; each device the library
// runs on holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address is looked up once per device with
// hipGetSymbolAddress while the library's context is created on it, and that
// address is what the launches take.  Layout of one call:
//   [0, 256)                       the argument record of the CCL launches
//   [256, 256 + 4 (w*h + 1))       union-find ids (id 0 = virtual node)
//   then, 256-aligned              the component list (when a count is asked)
// Every call on a device shares the array and leaves its contents behind;
// calls that overlap on one device race.
#include <mutex>

#include "rt_internal.h"

namespace rtseg {

static __device__ __align__(256) unsigned char scratch[RT_NOALLOC_SCRATCH_BYTES];
static_assert(sizeof(CclArgs) <= 256, "the argument record must fit the first 256 bytes");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

__global__ void k_put_ccl_args(CclArgs a, CclArgs *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

int noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("no-allocation scratch: device %d beyond the table of %d devices", device, kMaxDevices);
        return RT_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return RT_OK;
    void *p = nullptr;
    // the caller has made `device` current
    RT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("no-allocation scratch: hipGetSymbolAddress returned a null address");
        return RT_EDEVICE;
    }
    g_ptr[device] = p;
    return RT_OK;
}

size_t noalloc_ccl_bytes(int w, int h, int conn, bool want_count) {
    const size_t npx = (size_t)w * h;
    size_t b = 256 + al256(sizeof(int32_t) * (npx + 1)) + al256(sizeof(int32_t) * ccl_border_ints(w, h));
    if (want_count) b += al256(sizeof(int32_t) * max_components(w, h, conn));
    return b;
}

int ccl_noalloc(int device, int n_cu, const uint8_t *mask, int32_t *labels, int w, int h, int64_t pitch, int conn,
                int32_t *n_out_dev, hipStream_t s) {
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (device >= 0 && device < kMaxDevices) base = g_ptr[device];
    }
    if (!base) {
        set_error("rt_ccl_noalloc: no scratch address for device %d (create a context on it first)", device);
        return RT_EDEVICE;
    }
    const size_t need = noalloc_ccl_bytes(w, h, conn, n_out_dev != nullptr);
    if ((int64_t)w * h > RT_NOALLOC_MAX_PIXELS || need > (size_t)RT_NOALLOC_SCRATCH_BYTES) {
        set_error("rt_ccl_noalloc: %dx%d needs %zu bytes of scratch; the fixed array holds %d bytes for at most "
                  "%d pixels", w, h, need, RT_NOALLOC_SCRATCH_BYTES, RT_NOALLOC_MAX_PIXELS);
        return RT_EINVAL;
    }
    char *p = (char *)base;
    CclArgs *args = (CclArgs *)p;
    int32_t *ids = (int32_t *)(p + 256);
    int32_t *bt = (int32_t *)(p + 256 + al256(sizeof(int32_t) * ((size_t)w * h + 1)));
    int32_t *list = (int32_t *)((char *)bt + al256(sizeof(int32_t) * ccl_border_ints(w, h)));
    CclArgs A{};
    A.pred = CclPred::NonZero;
    A.out = CclOut::Labels;
    A.conn = conn;
    A.w = w;
    A.h = h;
    A.a = mask;
    A.pitch_a = pitch;
    A.ids = ids;
    A.bt = bt;
    A.labels = labels;
    A.pitch_l = pitch;
    if (n_out_dev) {
        A.obj_list = list;
        A.n_obj = n_out_dev;
        int e = launch_fill_i32(n_out_dev, 0, 1, s);
        if (e) return e;
    }
    hipLaunchKernelGGL(k_put_ccl_args, dim3(1), dim3(64), 0, s, A, args);
    RT_HIP(hipGetLastError());
    return launch_ccl(args, 1, ccl_tiles(w, h), n_cu, s, CclPred::NonZero, CclOut::Labels);
}

}  // namespace rtseg
