// Address arithmetic of the per-object crop loads, shared by the kernels and
// the host-side bounds check of the test suite (which compiles this header
// for the host and walks every load of every component of its inputs).
//
// A component's crop is its bounding box grown by one pixel, clipped to the
// image.  The crop is held in a plane of `st` columns per row (st >= cw: odd
// for the LDS classes, R + 1 for the register classes), so plane entries
// with column c >= cw lie outside the crop.  Loads are issued in batches of
// LOADS_IN_FLIGHT per thread: entry i of the plane is loaded by thread
// (i - i0) % nthreads of batch i0.  Every load address is clamped into the
// crop -- the plane index to the last entry, its column to the crop width --
// so the batch can issue all its loads before testing any of them; the
// padding columns and the entries past the plane's end are discarded after
// the load.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rtseg {

constexpr int LOADS_IN_FLIGHT = 8;

struct CropGeom {
    int cx0, cy0, cw, ch, st, n;
};

// crop of the component with bounding box [x0, x1] x [y0, y1] in a w x h
// image, plane stride cw | 1
__host__ __device__ inline CropGeom crop_of_box(int x0, int y0, int x1, int y1, int w, int h) {
    CropGeom q;
    q.cx0 = x0 - 1 > 0 ? x0 - 1 : 0;
    q.cy0 = y0 - 1 > 0 ? y0 - 1 : 0;
    const int cx1 = x1 + 1 < w - 1 ? x1 + 1 : w - 1, cy1 = y1 + 1 < h - 1 ? y1 + 1 : h - 1;
    q.cw = cx1 - q.cx0 + 1;
    q.ch = cy1 - q.cy0 + 1;
    q.st = q.cw | 1;
    q.n = q.st * q.ch;
    return q;
}

__host__ __device__ inline CropGeom crop_with_stride(CropGeom q, int st) {
    q.st = st;
    q.n = st * q.ch;
    return q;
}

// image offset (elements, row pitch `pitch`) loaded for plane entry i of the
// crop; i is clamped to [0, n - 1] and its column to [0, cw - 1]
__host__ __device__ inline int64_t crop_load_offset(const CropGeom &q, int i, int64_t pitch) {
    i = i < q.n - 1 ? i : q.n - 1;
    i = i > 0 ? i : 0;
    const int r = i / q.st;
    int c = i - r * q.st;
    c = c < q.cw - 1 ? c : q.cw - 1;
    c = c > 0 ? c : 0;
    return (int64_t)(q.cy0 + r) * pitch + q.cx0 + c;
}

// Dense order for the register classes (crops of at most 64 x 64): crop
// pixel k (raster order over the crop's cw x ch pixels, not over the plane)
// is row k / cw, column k - row cw, so a batch covers no padding column.  The
// quotient is (k + 1/2) (1 / cw) rounded down in single precision: with
// k < 4096 and cw <= 64 the rounding error of the two operations stays below
// 1e-3 while (k + 1/2) / cw lies at least 1 / 128 from an integer, so the
// result is exact (the host test also checks every k and cw of that range).
__host__ __device__ inline int crop_dense_row(int k, float inv_cw) { return (int)(((float)k + 0.5f) * inv_cw); }

// image offset loaded for crop pixel k, k clamped to [0, cw ch - 1]; inv_cw = 1.0f / cw
__host__ __device__ inline int64_t crop_load_offset_dense(const CropGeom &q, int k, float inv_cw, int64_t pitch) {
    const int last = q.cw * q.ch - 1;
    k = k < last ? k : last;
    k = k > 0 ? k : 0;
    const int r = crop_dense_row(k, inv_cw);
    return (int64_t)(q.cy0 + r) * pitch + q.cx0 + (k - r * q.cw);
}

// Loads of the erase pass (one wave per component, lane = crop column c < cw,
// rows in batches of eight): row r clamped to the crop's last row.
__host__ __device__ inline int64_t crop_erase_offset(const CropGeom &q, int c, int r, int64_t pitch) {
    r = r < q.ch - 1 ? r : q.ch - 1;
    return (int64_t)(q.cy0 + r) * pitch + q.cx0 + c;
}

}  // namespace rtseg
