"""ctypes front end of the CPU oracle (``liboracle.so`` built from rt_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.
All arrays are numpy, C-contiguous, row-major, dense (pitch == width).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "rt_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "features_oracle.c"), os.path.join(_HERE, "morph_oracle.c"),
         os.path.join(_HERE, "stitch_oracle.c")]

DQ_MAX = 65535

# Ruifrok-Johnston H&E optical-density vectors; a zero third row means
# "normalize(H x E)".
STAIN_HE = np.array([0.650, 0.704, 0.286,
                     0.072, 0.990, 0.105,
                     0.0, 0.0, 0.0], dtype=np.float64)

DEFAULTS = dict(scale=85.0, t_fg=16, min_area=20, max_area=1000, h_seed=3)


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (plain -O2, no FP contraction)."""
    newest = max(os.path.getmtime(p) for p in _SRCS + [os.path.join(_HERE, "rt_oracle.h")])
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", _SO, *_SRCS, "-lm"])
    return _SO


def build_native(outdir: str) -> str:
    """Compiles the same source for timing on this host: -O3 -march=native,
    still without FP contraction (so the arithmetic is unchanged).  Built
    where it runs, never shipped: -march=native is only valid on this CPU."""
    so = os.path.join(outdir, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, *_SRCS,
                           "-lm"])
    return so


_lib = None
_so_override = None


def use_library(path: str) -> None:
    """Makes later calls load `path` (a build of rt_oracle.c) instead of the default build."""
    global _lib, _so_override
    _lib = None
    _so_override = path


def lib():
    global _lib
    if _lib is None:
        if _so_override:
            so = _so_override
        else:
            build()
            so = _SO
        L = C.CDLL(so)
        u8p = C.POINTER(C.c_uint8)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        f64p = C.POINTER(C.c_double)
        L.or_deconv.argtypes = [u8p, C.c_int, C.c_int, f64p, C.c_double, f64p, u8p]
        L.or_deconv_od.argtypes = [f64p, f64p, f64p]
        L.or_recon.argtypes = [i32p, i32p, u8p, C.c_int, C.c_int, C.c_int, i32p]
        L.or_fill_holes.argtypes = [u8p, C.c_int, C.c_int, C.c_int, u8p]
        L.or_ccl.argtypes = [u8p, C.c_int, C.c_int, C.c_int, i32p]
        L.or_area_filter.argtypes = [i32p, C.c_int, C.c_int, C.c_int, C.c_int, i32p, u8p]
        L.or_edt_sq.argtypes = [u8p, C.c_int, C.c_int, i64p]
        L.or_isqrt.argtypes = [C.c_int64]
        L.or_isqrt.restype = C.c_int64
        L.or_dq.argtypes = [u8p, C.c_int, C.c_int, i32p]
        L.or_watershed.argtypes = [u8p, u8p, C.c_int, C.c_int, C.c_int, i32p, u8p, i32p, i32p, i32p, i32p]
        L.or_segment_from_hq.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         u8p, i32p, u8p, u8p, u8p, u8p]
        L.or_stitch_from_hq.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        C.c_int, i32p, u8p]
        L.or_erode.argtypes = [u8p, C.c_int, C.c_int, C.c_int, u8p]
        L.or_dilate.argtypes = [u8p, C.c_int, C.c_int, C.c_int, u8p]
        L.or_open.argtypes = [u8p, C.c_int, C.c_int, C.c_int, u8p]
        L.or_recon_to_nuclei.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, u8p, u8p]
        L.or_rbc_detect.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int, u8p]
        L.or_sobel_mag.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_sobel_mag.restype = C.c_int64
        L.or_features.argtypes = [i32p, u8p, C.c_int, C.c_int, C.c_int, i32p, f64p, i64p]
        _lib = L
    return _lib


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def deconv(rgb, stain=STAIN_HE, scale=85.0, want_ch=False):
    rgb = _u8(rgb)
    h, w = rgb.shape[:2]
    hq = np.empty((h, w), np.uint8)
    ch = np.empty((h, w), np.float64) if want_ch else None
    st = np.ascontiguousarray(stain, np.float64)
    rc = lib().or_deconv(_p(rgb, C.c_uint8), w, h, _p(st, C.c_double), float(scale), _p(ch, C.c_double),
                         _p(hq, C.c_uint8))
    if rc:
        raise ValueError("singular stain matrix")
    return (hq, ch) if want_ch else hq


def deconv_od(od, stain=STAIN_HE):
    st = np.ascontiguousarray(stain, np.float64)
    o = np.ascontiguousarray(od, np.float64)
    out = np.zeros(1, np.float64)
    if lib().or_deconv_od(_p(st, C.c_double), _p(o, C.c_double), _p(out, C.c_double)):
        raise ValueError("singular stain matrix")
    return float(out[0])


def recon(marker, mask, domain=None, conn=8):
    mk = _i32(marker)
    ms = _i32(mask)
    h, w = ms.shape
    dm = _u8(domain) if domain is not None else None
    out = np.empty((h, w), np.int32)
    lib().or_recon(_p(mk, C.c_int32), _p(ms, C.c_int32), _p(dm, C.c_uint8), w, h, conn, _p(out, C.c_int32))
    return out


def fill_holes(binary, bg_conn=4):
    b = _u8(binary)
    h, w = b.shape
    out = np.empty((h, w), np.uint8)
    lib().or_fill_holes(_p(b, C.c_uint8), w, h, bg_conn, _p(out, C.c_uint8))
    return out


def ccl(binary, conn=8):
    b = _u8(binary)
    h, w = b.shape
    out = np.empty((h, w), np.int32)
    n = lib().or_ccl(_p(b, C.c_uint8), w, h, conn, _p(out, C.c_int32))
    return out, int(n)


def area_filter(labels, min_area, max_area):
    lab = _i32(labels)
    h, w = lab.shape
    out = np.empty((h, w), np.int32)
    mask = np.empty((h, w), np.uint8)
    k = lib().or_area_filter(_p(lab, C.c_int32), w, h, int(min_area), int(max_area), _p(out, C.c_int32),
                             _p(mask, C.c_uint8))
    return out, mask, int(k)


def edt_sq(fg):
    b = _u8(fg)
    h, w = b.shape
    out = np.empty((h, w), np.int64)
    lib().or_edt_sq(_p(b, C.c_uint8), w, h, _p(out, C.c_int64))
    return out


def isqrt(n: int) -> int:
    return int(lib().or_isqrt(int(n)))


def dq(fg):
    b = _u8(fg)
    h, w = b.shape
    out = np.empty((h, w), np.int32)
    lib().or_dq(_p(b, C.c_uint8), w, h, _p(out, C.c_int32))
    return out


def watershed(fg, seeds=None, h_seed=3, intermediates=False):
    b = _u8(fg)
    h, w = b.shape
    sd = _u8(seeds) if seeds is not None else None
    lab = np.empty((h, w), np.int32)
    mask = np.empty((h, w), np.uint8)
    if intermediates:
        dqa = np.empty((h, w), np.int32)
        sl = np.empty((h, w), np.int32)
        lam = np.empty((h, w), np.int32)
        fl = np.empty((h, w), np.int32)
    else:
        dqa = sl = lam = fl = None
    lib().or_watershed(_p(b, C.c_uint8), _p(sd, C.c_uint8), int(h_seed), w, h, _p(lab, C.c_int32),
                       _p(mask, C.c_uint8), _p(dqa, C.c_int32), _p(sl, C.c_int32), _p(lam, C.c_int32),
                       _p(fl, C.c_int32))
    if intermediates:
        return lab, mask, dict(dq=dqa, seeds=sl, lam=lam, flood=fl)
    return lab, mask


def segment_from_hq(hq, t_fg=16, min_area=20, max_area=1000, h_seed=3, intermediates=False):
    q = _u8(hq)
    h, w = q.shape
    mask = np.empty((h, w), np.uint8)
    lab = np.empty((h, w), np.int32)
    if intermediates:
        R = np.empty((h, w), np.uint8)
        F0 = np.empty((h, w), np.uint8)
        F = np.empty((h, w), np.uint8)
        A = np.empty((h, w), np.uint8)
    else:
        R = F0 = F = A = None
    n = lib().or_segment_from_hq(_p(q, C.c_uint8), w, h, int(t_fg), int(min_area), int(max_area), int(h_seed),
                                 _p(mask, C.c_uint8), _p(lab, C.c_int32), _p(R, C.c_uint8), _p(F0, C.c_uint8),
                                 _p(F, C.c_uint8), _p(A, C.c_uint8))
    if intermediates:
        return mask, lab, int(n), dict(R=R, F0=F0, F=F, A=A)
    return mask, lab, int(n)


def segment_rgb(rgb, stain=STAIN_HE, scale=85.0, **kw):
    """Whole plain pipeline from RGB: deconvolution, then segment_from_hq."""
    hq = deconv(rgb, stain, scale)
    mask, lab, n = segment_from_hq(hq, **kw)
    return hq, mask, lab, n


# feature computation (rt_oracle.h): names in output order
FEATURE_NAMES = (
    "area", "perimeter", "centroid_x", "centroid_y", "bbox_w", "bbox_h", "extent", "equiv_diameter",
    "circularity", "major_axis", "minor_axis", "eccentricity", "orientation",
    "int_mean", "int_std", "int_min", "int_max", "int_median", "int_p25", "int_p75", "int_skewness",
    "int_kurtosis", "int_entropy", "int_energy", "int_range",
    "grad_mean", "grad_std", "grad_max", "grad_entropy", "grad_energy", "edge_fraction",
    "glcm_asm", "glcm_contrast", "glcm_correlation", "glcm_variance", "glcm_homogeneity",
    "glcm_sum_average", "glcm_sum_variance", "glcm_sum_entropy", "glcm_entropy", "glcm_diff_variance",
    "glcm_diff_entropy", "glcm_imc1", "glcm_imc2", "glcm_max_prob", "glcm_cluster_shade",
    "glcm_cluster_prominence")
NFEAT = len(FEATURE_NAMES)
NCOUNT = 537
GLCM_LEVELS = 16
GRAD_BINS = 16
GRAD_BIN_WIDTH = 32
EDGE_THRESHOLD = 128


def sobel_mag(hq, x, y):
    q = _u8(hq)
    h, w = q.shape
    return int(lib().or_sobel_mag(_p(q, C.c_uint8), w, h, int(x), int(y)))


def features(labels, hq, want_counts=False):
    """Per-nucleus features.  Returns (labels [n] int32, feats [n, NFEAT]
    float64) and, with want_counts, the counts [n, NCOUNT] int64."""
    lab = _i32(labels)
    q = _u8(hq)
    h, w = lab.shape
    # the number of nuclei is at most the number of distinct positive labels
    cap = max(1, int(np.unique(lab[lab > 0]).size))
    lo = np.empty(cap, np.int32)
    fo = np.empty((cap, NFEAT), np.float64)
    co = np.empty((cap, NCOUNT), np.int64) if want_counts else None
    n = lib().or_features(_p(lab, C.c_int32), _p(q, C.c_uint8), w, h, cap, _p(lo, C.c_int32), _p(fo, C.c_double),
                          _p(co, C.c_int64))
    n = min(n, cap)
    if want_counts:
        return lo[:n], fo[:n], co[:n]
    return lo[:n], fo[:n]


# pre-processing operations (rt_oracle.h)
MARKER_FRAME = 0
MARKER_OPEN = 1


def _morph(fn, img, radius):
    a = _u8(img)
    h, w = a.shape
    out = np.empty((h, w), np.uint8)
    fn(_p(a, C.c_uint8), w, h, int(radius), _p(out, C.c_uint8))
    return out


def erode(img, radius):
    return _morph(lib().or_erode, img, radius)


def dilate(img, radius):
    return _morph(lib().or_dilate, img, radius)


def open_(img, radius):
    return _morph(lib().or_open, img, radius)


def recon_to_nuclei(hq, marker=MARKER_FRAME, radius=0, t_fg=16):
    """Returns (R, F0)."""
    q = _u8(hq)
    h, w = q.shape
    r = np.empty((h, w), np.uint8)
    f0 = np.empty((h, w), np.uint8)
    lib().or_recon_to_nuclei(_p(q, C.c_uint8), w, h, int(marker), int(radius), int(t_fg), _p(r, C.c_uint8),
                             _p(f0, C.c_uint8))
    return r, f0


def rbc_detect(rgb, t_strong=200, t_weak=150):
    a = _u8(rgb)
    h, w = a.shape[:2]
    out = np.empty((h, w), np.uint8)
    lib().or_rbc_detect(_p(a, C.c_uint8), w, h, int(t_strong), int(t_weak), _p(out, C.c_uint8))
    return out


def stitch_from_hq(hq, tile, halo, t_fg=16, min_area=20, max_area=1000, h_seed=3):
    """Cross-tile stitching (rt_oracle.h): returns (labels, mask, n_owned)."""
    q = _u8(hq)
    H, W = q.shape
    lab = np.empty((H, W), np.int32)
    mask = np.empty((H, W), np.uint8)
    n = lib().or_stitch_from_hq(_p(q, C.c_uint8), W, H, int(tile), int(halo), int(t_fg), int(min_area),
                                int(max_area), int(h_seed), _p(lab, C.c_int32), _p(mask, C.c_uint8))
    return lab, mask, int(n)
