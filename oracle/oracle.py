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

DQ_MAX = 65535

# Ruifrok-Johnston H&E optical-density vectors; a zero third row means
# "normalize(H x E)".
STAIN_HE = np.array([0.650, 0.704, 0.286,
                     0.072, 0.990, 0.105,
                     0.0, 0.0, 0.0], dtype=np.float64)

DEFAULTS = dict(scale=85.0, t_fg=16, min_area=20, max_area=1000, h_seed=3)


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"])
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
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
