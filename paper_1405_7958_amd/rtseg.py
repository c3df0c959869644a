"""Python binding of librtseg.so (C ABI in include/rtseg.h).

Argument marshalling only: every step of the segmentation runs in the HIP
kernels of librtseg.so.  Tensors must be HIP device tensors (torch ``cuda``
tensors on ROCm) of the stated dtype; 2-D images may be row-pitched (last
stride 1).  Calls are enqueued on torch's current stream.  If the library is
not built, every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtseg.so")

RT_OK = 0
RT_EINVAL = -1
RT_ENOMEM = -2
RT_EDEVICE = -3
RT_EUNSUPPORTED = -4
RT_U8 = 1
RT_I32 = 2
DQ_MAX = 65535


class RtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtseg error {code}: {msg}")
        self.code = code


class rt_seg_params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("stain_rows", C.c_double * 9), ("hq_scale", C.c_double),
                ("t_fg", C.c_int32), ("min_area", C.c_int32), ("max_area", C.c_int32),
                ("h_seed", C.c_int32), ("conn", C.c_int32)]


class rt_host_tile(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("rgb_pitch_bytes", C.c_int64), ("w", C.c_int32), ("h", C.c_int32),
                ("mask", C.c_void_p), ("labels", C.c_void_p), ("out_pitch", C.c_int64), ("n_objects", C.c_void_p)]


class rt_tile_desc(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("rgb_pitch_bytes", C.c_int64), ("w", C.c_int32), ("h", C.c_int32),
                ("mask_out", C.c_void_p), ("labels_out", C.c_void_p), ("out_pitch", C.c_int64),
                ("n_objects_dev", C.c_void_p), ("hq_out", C.c_void_p), ("fg_out", C.c_void_p),
                ("seeds_out", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.rt_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.rt_ctx_destroy.argtypes = [vp]
        L.rt_last_error.restype = C.c_char_p
        L.rt_sync.argtypes = [vp, vp]
        L.rt_deconv.argtypes = [vp, vp, i64, i32, i32, C.POINTER(C.c_double), C.c_double, vp, i64, vp, i64, vp]
        L.rt_morph_recon.argtypes = [vp, C.c_int, vp, vp, vp, vp, i32, i32, i64, C.c_int, vp]
        L.rt_fill_holes.argtypes = [vp, vp, vp, i32, i32, i64, C.c_int, vp]
        L.rt_ccl.argtypes = [vp, vp, vp, i32, i32, i64, C.c_int, vp, vp]
        L.rt_ccl_noalloc.argtypes = [vp, vp, vp, i32, i32, i64, C.c_int, vp, vp]
        L.rt_features.argtypes = [vp, vp, i64, vp, i64, i32, i32, i32, vp, vp, vp, vp, vp]
        L.rt_morph.argtypes = [vp, C.c_int, vp, i64, vp, i64, i32, i32, i32, vp]
        L.rt_recon_to_nuclei.argtypes = [vp, vp, vp, vp, i32, i32, i64, C.c_int, i32, i32, vp]
        L.rt_rbc_detect.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp, i64, vp]
        L.rt_area_filter.argtypes = [vp, vp, vp, vp, i32, i32, i64, i32, i32, vp]
        L.rt_watershed.argtypes = [vp, vp, vp, i32, vp, vp, i32, i32, i64, vp]
        L.rt_seg_params_default.argtypes = [C.POINTER(rt_seg_params)]
        L.rt_segment_tile.argtypes = [vp, vp, i64, i32, i32, C.POINTER(rt_seg_params), vp, vp, i64, vp, vp, vp]
        L.rt_segment_batch.argtypes = [vp, i32, C.POINTER(rt_tile_desc), C.POINTER(rt_seg_params), vp]
        L.rt_segment_host_stream.argtypes = [vp, i32, C.POINTER(rt_host_tile), C.POINTER(rt_seg_params), i32, vp]
        L.rt_segment_slide.argtypes = [vp, vp, i64, i32, i32, i32, i32, C.POINTER(rt_seg_params), vp, vp, i64, vp,
                                       vp, vp]
        L.rt_set_knob.argtypes = [vp, C.c_char_p, C.c_int]
        L.rt_get_knob.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int)]
        L.rt_profile_enable.argtypes = [vp, C.c_int]
        L.rt_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
        u64 = C.c_uint64
        f32 = C.c_float
        L.rt_unet_param_count.restype = C.c_int64
        L.rt_unet_param_count.argtypes = []
        L.rt_unet_create.argtypes = [vp, u64, C.POINTER(vp)]
        L.rt_unet_destroy.argtypes = [vp]
        L.rt_unet_get_params.argtypes = [vp, vp, i64]
        L.rt_unet_set_params.argtypes = [vp, vp, i64]
        L.rt_unet_get_grads.argtypes = [vp, vp, i64]
        L.rt_unet_grad_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, f32, vp, vp]
        L.rt_unet_train_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, f32, f32, vp, vp]
        L.rt_unet_forward.argtypes = [vp, vp, i64, i32, i32, vp, vp, i64, vp]
        L.rt_unet_save.argtypes = [vp, C.c_char_p]
        L.rt_unet_load.argtypes = [vp, C.c_char_p]
        L.rt_unet_adam_step.argtypes = [vp, f32, vp]
        L.rt_unet_get_step.argtypes = [vp, C.POINTER(i64)]
        L.rt_unet_save_checkpoint.argtypes = [vp, C.c_char_p]
        L.rt_unet_load_checkpoint.argtypes = [vp, C.c_char_p]
        L.rt_segment_tile_surrogate.argtypes = [vp, vp, vp, i64, i32, i32, C.POINTER(rt_seg_params), f32, vp, vp,
                                                i64, vp, C.POINTER(C.c_int32), C.POINTER(C.c_float), vp]
        L.rt_nn_conv3_fwd.argtypes = [vp, vp, i32, vp, i32, i32, i32, i32, vp, vp, i32, i32, vp, vp, vp]
        L.rt_nn_conv3_dgrad.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, i32, vp, vp, vp]
        L.rt_nn_conv3_wgrad.argtypes = [vp, vp, i32, vp, i32, vp, i32, i32, i32, i32, vp, vp, vp]
        L.rt_nn_up2_fwd.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, i32, vp, vp, vp]
        L.rt_nn_up2_bwd.argtypes = [vp, vp, i32, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.rt_nn_pool2.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.rt_nn_head_loss.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp]
        L.rt_nn_pack.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp]
        L.rt_nn_prep_input.argtypes = [vp, vp, i64, i32, i32, vp, vp]
        L.rt_profile_recon_rounds.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.rt_profile_objects.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]
        L.rt_profile_stage_name.argtypes = [C.c_int]
        L.rt_profile_stage_name.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != RT_OK:
        raise RtError(rc, lib().rt_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _img(t, dtype, name, channels=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if channels is None:
        if t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{name}: expected a 2-D row-major image")
    else:
        if t.dim() != 3 or t.shape[2] != channels or t.stride(2) != 1 or t.stride(1) != channels:
            raise ValueError(f"{name}: expected an (H, W, {channels}) interleaved image")
    return t


class Context:
    """Owns an rt_ctx (scratch memory) on one device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = C.c_void_p()
        _check(lib().rt_ctx_create(device, C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().rt_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(lib().rt_sync(self.h, _stream()))


_default = {}


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def default_params(**over):
    p = rt_seg_params()
    lib().rt_seg_params_default(C.byref(p))
    for k, v in over.items():
        if k == "stain_rows":
            for i in range(9):
                p.stain_rows[i] = float(v[i])
        else:
            setattr(p, k, v)
    return p


STAIN_HE = (0.650, 0.704, 0.286, 0.072, 0.990, 0.105, 0.0, 0.0, 0.0)


def rt_deconv(rgb, stain=STAIN_HE, hq_scale=85.0, want_ch=False, ctx=None, hq_out=None):
    ctx = ctx or default_context(rgb.device.index)
    _img(rgb, torch.uint8, "rgb", 3)
    h, w = rgb.shape[:2]
    hq = hq_out if hq_out is not None else torch.empty((h, w), dtype=torch.uint8, device=rgb.device)
    ch = torch.empty((h, w), dtype=torch.float32, device=rgb.device) if want_ch else None
    st = (C.c_double * 9)(*[float(v) for v in stain])
    _check(lib().rt_deconv(ctx.h, _ptr(rgb), rgb.stride(0), w, h, st, float(hq_scale), _ptr(ch),
                           ch.stride(0) if ch is not None else 0, _ptr(hq), hq.stride(0), _stream()))
    return (hq, ch) if want_ch else hq


def rt_morph_recon(marker, mask, domain=None, conn=8, out=None, ctx=None):
    ctx = ctx or default_context(mask.device.index)
    if mask.dtype == torch.uint8:
        dt = RT_U8
    elif mask.dtype == torch.int32:
        dt = RT_I32
    else:
        raise TypeError("rt_morph_recon: uint8 or int32 images")
    _img(mask, mask.dtype, "mask")
    _img(marker, mask.dtype, "marker")
    if marker.shape != mask.shape or marker.stride(0) != mask.stride(0):
        raise ValueError("marker and mask must share shape and pitch")
    if domain is not None:
        _img(domain, torch.uint8, "domain")
        if domain.shape != mask.shape or domain.stride(0) != mask.stride(0):
            raise ValueError("domain must share shape and pitch with mask")
    h, w = mask.shape
    if out is None:
        out = torch.empty_strided(mask.shape, mask.stride(), dtype=mask.dtype, device=mask.device)
    _check(lib().rt_morph_recon(ctx.h, dt, _ptr(marker), _ptr(mask), _ptr(out), _ptr(domain), w, h,
                                mask.stride(0), conn, _stream()))
    return out


def rt_fill_holes(binary, bg_conn=4, out=None, ctx=None):
    ctx = ctx or default_context(binary.device.index)
    _img(binary, torch.uint8, "binary")
    h, w = binary.shape
    if out is None:
        out = torch.empty_strided(binary.shape, binary.stride(), dtype=torch.uint8, device=binary.device)
    _check(lib().rt_fill_holes(ctx.h, _ptr(binary), _ptr(out), w, h, binary.stride(0), bg_conn, _stream()))
    return out


def rt_ccl(binary, conn=8, ctx=None):
    """Returns (labels int32, n_components as a 1-element device tensor)."""
    ctx = ctx or default_context(binary.device.index)
    _img(binary, torch.uint8, "binary")
    h, w = binary.shape
    lab = torch.empty_strided(binary.shape, binary.stride(), dtype=torch.int32, device=binary.device)
    n = torch.zeros(1, dtype=torch.int32, device=binary.device)
    _check(lib().rt_ccl(ctx.h, _ptr(binary), _ptr(lab), w, h, binary.stride(0), conn, _ptr(n), _stream()))
    return lab, n


def rt_ccl_noalloc(binary, labels, n_out=None, conn=8, ctx=None):
    """rt_ccl with the library's fixed device scratch array: writes into the
    caller's `labels` (int32, same shape and pitch as `binary`) and, when
    given, the 1-element int32 device tensor `n_out`; allocates nothing."""
    ctx = ctx or default_context(binary.device.index)
    _img(binary, torch.uint8, "binary")
    _img(labels, torch.int32, "labels")
    if labels.shape != binary.shape or labels.stride(0) != binary.stride(0):
        raise ValueError("labels must share shape and pitch with binary")
    if n_out is not None and (n_out.dtype != torch.int32 or not n_out.is_cuda or n_out.numel() < 1):
        raise ValueError("n_out must be an int32 device tensor")
    h, w = binary.shape
    _check(lib().rt_ccl_noalloc(ctx.h, _ptr(binary), _ptr(labels), w, h, binary.stride(0), conn,
                                _ptr(n_out) if n_out is not None else None, _stream()))
    return labels, n_out


RT_ERODE, RT_DILATE, RT_OPEN = 0, 1, 2
RT_MARKER_FRAME, RT_MARKER_OPEN = 0, 1
RT_MORPH_MAX_RADIUS = 32


def rt_morph(img, op, radius, ctx=None):
    """Grey erosion / dilation / opening by the flat disk of `radius`."""
    ctx = ctx or default_context(img.device.index)
    _img(img, torch.uint8, "img")
    h, w = img.shape
    out = torch.empty((h, w), dtype=torch.uint8, device=img.device)
    _check(lib().rt_morph(ctx.h, int(op), _ptr(img), img.stride(0), _ptr(out), w, w, h, int(radius), _stream()))
    return out


def rt_recon_to_nuclei(hq, marker=RT_MARKER_FRAME, radius=0, t_fg=16, ctx=None):
    """Returns (R, F0) of ReconToNuclei with the frame or opening-by-
    reconstruction marker."""
    ctx = ctx or default_context(hq.device.index)
    _img(hq, torch.uint8, "hq")
    h, w = hq.shape
    r = torch.empty_strided(hq.shape, hq.stride(), dtype=torch.uint8, device=hq.device)
    f0 = torch.empty_strided(hq.shape, hq.stride(), dtype=torch.uint8, device=hq.device)
    _check(lib().rt_recon_to_nuclei(ctx.h, _ptr(hq), _ptr(r), _ptr(f0), w, h, hq.stride(0), int(marker),
                                    int(radius), int(t_fg), _stream()))
    return r, f0


def rt_rbc_detect(rgb, t_strong=200, t_weak=150, ctx=None):
    ctx = ctx or default_context(rgb.device.index)
    _img(rgb, torch.uint8, "rgb", 3)
    h, w = rgb.shape[:2]
    out = torch.empty((h, w), dtype=torch.uint8, device=rgb.device)
    _check(lib().rt_rbc_detect(ctx.h, _ptr(rgb), rgb.stride(0), w, h, int(t_strong), int(t_weak), _ptr(out), w,
                               _stream()))
    return out


RT_NFEAT = 47
RT_FEAT_NCOUNT = 537


def rt_features(labels, hq, max_nuclei=65536, want_counts=False, ctx=None):
    """Per-nucleus features (include/rtseg.h).  labels: int32 (H, W) with the
    segmentation's labels; hq: uint8 (H, W).  Returns (labels_out [n] int32,
    feats [n, RT_NFEAT] float64, counts [n, RT_FEAT_NCOUNT] int64 or None,
    n_total) with n = min(n_total, max_nuclei); reads the count back."""
    ctx = ctx or default_context(labels.device.index)
    _img(labels, torch.int32, "labels")
    _img(hq, torch.uint8, "hq")
    if labels.shape != hq.shape:
        raise ValueError("labels and hq must have the same shape")
    h, w = labels.shape
    d = labels.device
    m = int(max_nuclei)
    lo = torch.empty(max(m, 1), dtype=torch.int32, device=d)
    fo = torch.empty((max(m, 1), RT_NFEAT), dtype=torch.float64, device=d)
    co = torch.empty((max(m, 1), RT_FEAT_NCOUNT), dtype=torch.int64, device=d) if want_counts else None
    n = torch.zeros(1, dtype=torch.int32, device=d)
    _check(lib().rt_features(ctx.h, _ptr(labels), labels.stride(0), _ptr(hq), hq.stride(0), w, h, m, _ptr(lo),
                             _ptr(fo), _ptr(co), _ptr(n), _stream()))
    total = int(n.item())
    k = min(total, m)
    return lo[:k], fo[:k], (co[:k] if co is not None else None), total


def rt_area_filter(labels, min_area, max_area, ctx=None):
    ctx = ctx or default_context(labels.device.index)
    _img(labels, torch.int32, "labels")
    h, w = labels.shape
    out = torch.empty_strided(labels.shape, labels.stride(), dtype=torch.int32, device=labels.device)
    mask = torch.empty_strided(labels.shape, labels.stride(), dtype=torch.uint8, device=labels.device)
    _check(lib().rt_area_filter(ctx.h, _ptr(labels), _ptr(out), _ptr(mask), w, h, labels.stride(0),
                                int(min_area), int(max_area), _stream()))
    return out, mask


def rt_watershed(fg, seeds=None, h_seed=3, ctx=None):
    ctx = ctx or default_context(fg.device.index)
    _img(fg, torch.uint8, "fg")
    if seeds is not None:
        _img(seeds, torch.uint8, "seeds")
        if seeds.shape != fg.shape or seeds.stride(0) != fg.stride(0):
            raise ValueError("seeds must share shape and pitch with fg")
    h, w = fg.shape
    lab = torch.empty_strided(fg.shape, fg.stride(), dtype=torch.int32, device=fg.device)
    mask = torch.empty_strided(fg.shape, fg.stride(), dtype=torch.uint8, device=fg.device)
    _check(lib().rt_watershed(ctx.h, _ptr(fg), _ptr(seeds), int(h_seed), _ptr(lab), _ptr(mask), w, h,
                              fg.stride(0), _stream()))
    return lab, mask


def rt_segment_tile(rgb, params=None, want_hq=False, ctx=None, out=None):
    """Returns (mask uint8, labels int32, n_objects 1-element device tensor[, hq])."""
    ctx = ctx or default_context(rgb.device.index)
    _img(rgb, torch.uint8, "rgb", 3)
    h, w = rgb.shape[:2]
    p = params if params is not None else default_params()
    if out is None:
        mask = torch.empty((h, w), dtype=torch.uint8, device=rgb.device)
        lab = torch.empty((h, w), dtype=torch.int32, device=rgb.device)
        n = torch.zeros(1, dtype=torch.int32, device=rgb.device)
        hq = torch.empty((h, w), dtype=torch.uint8, device=rgb.device) if want_hq else None
    else:
        mask, lab, n, hq = out
    _check(lib().rt_segment_tile(ctx.h, _ptr(rgb), rgb.stride(0), w, h, C.byref(p), _ptr(mask), _ptr(lab),
                                 lab.stride(0), _ptr(n), _ptr(hq), _stream()))
    return (mask, lab, n, hq) if want_hq else (mask, lab, n)


def rt_segment_batch(rgbs, params=None, want_hq=False, ctx=None, want_maps=False):
    """Segments a list of (H_i, W_i, 3) uint8 device tiles in one call.

    Returns a list of (mask, labels, n_objects[, hq][, fg, seeds]) per tile,
    as rt_segment_tile would for each tile alone; with want_maps the
    foreground after the first area threshold and its watershed seeds are
    returned too (uint8 0/1 maps)."""
    ctx = ctx or (default_context(rgbs[0].device.index) if rgbs else default_context())
    p = params if params is not None else default_params()
    outs = []
    descs = (rt_tile_desc * max(1, len(rgbs)))()
    for i, rgb in enumerate(rgbs):
        _img(rgb, torch.uint8, f"rgbs[{i}]", 3)
        h, w = rgb.shape[:2]
        mask = torch.empty((h, w), dtype=torch.uint8, device=rgb.device)
        lab = torch.empty((h, w), dtype=torch.int32, device=rgb.device)
        n = torch.zeros(1, dtype=torch.int32, device=rgb.device)
        hq = torch.empty((h, w), dtype=torch.uint8, device=rgb.device) if want_hq else None
        fg = torch.empty((h, w), dtype=torch.uint8, device=rgb.device) if want_maps else None
        sd = torch.empty((h, w), dtype=torch.uint8, device=rgb.device) if want_maps else None
        descs[i] = rt_tile_desc(rgb.data_ptr(), rgb.stride(0), w, h, mask.data_ptr(), lab.data_ptr(), w,
                                n.data_ptr(), hq.data_ptr() if hq is not None else None,
                                fg.data_ptr() if fg is not None else None, sd.data_ptr() if sd is not None else None)
        o = (mask, lab, n, hq) if want_hq else (mask, lab, n)
        outs.append(o + (fg, sd) if want_maps else o)
    _check(lib().rt_segment_batch(ctx.h, len(rgbs), descs, C.byref(p), _stream()))
    return outs


RT_PROF_STAGES = 7
KNOBS = ("recon_levels", "recon_level_mode", "recon_level_frac", "recon_round_batch", "recon_max_sweeps", "recon_mode",
         "recon_queue_after", "objects_path", "graph", "graph_rounds", "recon_async", "recon_async_rounds",
         "objects_streams")
READ_ONLY = ("graph_captures", "graph_replays", "last_rounds", "recon_host_reads")


def rt_segment_slide(rgb, tile, halo, params=None, want_hq=False, ctx=None):
    """Cross-tile stitching of a device slide (H, W, 3): returns (labels,
    mask, n_objects[, hq])."""
    ctx = ctx or default_context(rgb.device.index)
    _img(rgb, torch.uint8, "rgb", 3)
    p = params or default_params()
    H, W = rgb.shape[:2]
    d = rgb.device
    lab = torch.empty((H, W), dtype=torch.int32, device=d)
    mask = torch.empty((H, W), dtype=torch.uint8, device=d)
    hq = torch.empty((H, W), dtype=torch.uint8, device=d) if want_hq else None
    n = torch.zeros(1, dtype=torch.int32, device=d)
    _check(lib().rt_segment_slide(ctx.h, _ptr(rgb), rgb.stride(0), W, H, int(tile), int(halo), C.byref(p), _ptr(lab),
                                  _ptr(mask), W, _ptr(hq), _ptr(n), _stream()))
    return (lab, mask, n, hq) if want_hq else (lab, mask, n)


def rt_segment_host_stream(rgbs, params=None, depth=3, want_mask=True, want_labels=True, ctx=None, outs=None):
    """Segments host-resident tiles (CPU uint8 tensors (H, W, 3), ideally
    pinned) with uploads, computation and downloads overlapped; results in
    pinned host tensors: a list of (mask, labels, n_objects) (None where not
    wanted).  `outs` (optional) reuses the output tensors of an earlier call."""
    ctx = ctx or default_context()
    p = params or default_params()
    n = len(rgbs)
    descs = (rt_host_tile * max(n, 1))()
    res = []
    for i, t in enumerate(rgbs):
        if t.is_cuda or t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3 or t.stride(2) != 1 \
                or t.stride(1) != 3:
            raise ValueError(f"tile {i}: expected a host (H, W, 3) uint8 interleaved tensor")
        h, w = t.shape[:2]
        if outs is not None:
            m, lab, cnt = outs[i]
        else:
            m = torch.empty((h, w), dtype=torch.uint8, pin_memory=True) if want_mask else None
            lab = torch.empty((h, w), dtype=torch.int32, pin_memory=True) if want_labels else None
            cnt = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        descs[i] = rt_host_tile(t.data_ptr(), t.stride(0), w, h, m.data_ptr() if m is not None else None,
                                lab.data_ptr() if lab is not None else None, w, cnt.data_ptr())
        res.append((m, lab, cnt))
    _check(lib().rt_segment_host_stream(ctx.h, n, descs, C.byref(p), int(depth), _stream()))
    return res


def rt_set_knob(name, value, ctx=None):
    ctx = ctx or default_context()
    _check(lib().rt_set_knob(ctx.h, name.encode(), int(value)))


def rt_get_knob(name, ctx=None):
    ctx = ctx or default_context()
    v = C.c_int()
    _check(lib().rt_get_knob(ctx.h, name.encode(), C.byref(v)))
    return v.value



def rt_profile_enable(enable=True, ctx=None):
    """True / 1: stage and round timing; 2: round timing only; False / 0: off."""
    ctx = ctx or default_context()
    mode = 1 if enable is True else int(enable)
    if mode not in (0, 1, 2):
        raise ValueError("rt_profile_enable: 0, 1 or 2")
    _check(lib().rt_profile_enable(ctx.h, mode))


def rt_profile_read(ctx=None):
    """Returns (n_calls, {stage: (ms_total, launches)}) since the last read."""
    ctx = ctx or default_context()
    ms = (C.c_double * RT_PROF_STAGES)()
    ln = (C.c_int64 * RT_PROF_STAGES)()
    n = lib().rt_profile_read(ctx.h, ms, ln, RT_PROF_STAGES)
    if n < 0:
        _check(n)
    names = [lib().rt_profile_stage_name(i).decode() for i in range(RT_PROF_STAGES)]
    return n, {names[i]: (ms[i], int(ln[i])) for i in range(RT_PROF_STAGES)}


def rt_profile_objects(cls, ctx=None):
    """Returns (kernel_ms, launches, component_pixels) of per-object class
    `cls` (0 small, 1 medium, 2 large) since the last read."""
    ctx = ctx or default_context()
    ms = C.c_double()
    ln = C.c_int64()
    px = C.c_int64()
    _check(lib().rt_profile_objects(ctx.h, int(cls), C.byref(ms), C.byref(ln), C.byref(px)))
    return ms.value, ln.value, px.value


def rt_profile_recon_rounds(ctx=None):
    """Returns (kernel_ms, launches, tile_visits) of the reconstruction round
    kernel since the last read (recorded in profiling modes 1 and 2)."""
    ctx = ctx or default_context()
    ms = C.c_double()
    ln = C.c_int64()
    tv = C.c_int64()
    _check(lib().rt_profile_recon_rounds(ctx.h, C.byref(ms), C.byref(ln), C.byref(tv)))
    return ms.value, ln.value, tv.value


# ----------------------------------------------------------------------------
# the U-Net surrogate (include/rtseg_unet.h)
# ----------------------------------------------------------------------------

def unet_param_count():
    return int(lib().rt_unet_param_count())


class UNet:
    """Owns an rt_unet on the context's device."""

    def __init__(self, seed: int = 0, ctx=None):
        self.ctx = ctx or default_context()
        h = C.c_void_p()
        _check(lib().rt_unet_create(self.ctx.h, C.c_uint64(seed), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().rt_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.empty(unet_param_count(), np.float32)
        _check(lib().rt_unet_get_params(self.h, out.ctypes.data, out.size))
        return out

    def set_params(self, vec):
        import numpy as np
        v = np.ascontiguousarray(vec, dtype=np.float32)
        _check(lib().rt_unet_set_params(self.h, v.ctypes.data, v.size))

    def get_grads(self):
        import numpy as np
        out = np.empty(unet_param_count(), np.float32)
        _check(lib().rt_unet_get_grads(self.h, out.ctypes.data, out.size))
        return out

    def _batch(self, rgb, fg, seed):
        _img(rgb[0], torch.uint8, "rgb[0]", 3)
        if not (rgb.is_contiguous() and fg.is_contiguous() and seed.is_contiguous()):
            raise ValueError("batch tensors must be contiguous")
        b, h, w = rgb.shape[:3]
        if fg.shape != (b, h, w) or seed.shape != (b, h, w) or fg.dtype != torch.uint8 or seed.dtype != torch.uint8:
            raise ValueError("targets must be (b, h, w) uint8")
        return b, h, w

    def grad_step(self, rgb, fg, seed, w_seed=1.0, loss=None):
        """Adds the gradient of the batch loss; returns the loss tensor (device)."""
        b, h, w = self._batch(rgb, fg, seed)
        loss = loss if loss is not None else torch.zeros(1, dtype=torch.float32, device=rgb.device)
        _check(lib().rt_unet_grad_step(self.h, _ptr(rgb), _ptr(fg), _ptr(seed), b, h, w, float(w_seed), _ptr(loss),
                                       _stream()))
        return loss

    def train_step(self, rgb, fg, seed, lr=1e-3, w_seed=1.0, loss=None):
        b, h, w = self._batch(rgb, fg, seed)
        loss = loss if loss is not None else torch.zeros(1, dtype=torch.float32, device=rgb.device)
        _check(lib().rt_unet_train_step(self.h, _ptr(rgb), _ptr(fg), _ptr(seed), b, h, w, float(lr), float(w_seed),
                                        _ptr(loss), _stream()))
        return loss

    def adam_step(self, lr=1e-3):
        """One Adam update from the accumulated gradient (then cleared)."""
        _check(lib().rt_unet_adam_step(self.h, float(lr), _stream()))

    @property
    def step(self):
        t = C.c_int64(0)
        _check(lib().rt_unet_get_step(self.h, C.byref(t)))
        return int(t.value)

    def save_checkpoint(self, path):
        _check(lib().rt_unet_save_checkpoint(self.h, os.fsencode(path)))

    def load_checkpoint(self, path):
        _check(lib().rt_unet_load_checkpoint(self.h, os.fsencode(path)))

    def forward(self, rgb):
        """(H, W, 3) uint8 tile -> (p_fg, p_seed) float32 maps."""
        _img(rgb, torch.uint8, "rgb", 3)
        h, w = rgb.shape[:2]
        pf = torch.empty((h, w), dtype=torch.float32, device=rgb.device)
        ps = torch.empty((h, w), dtype=torch.float32, device=rgb.device)
        _check(lib().rt_unet_forward(self.h, _ptr(rgb), rgb.stride(0), w, h, _ptr(pf), _ptr(ps), w, _stream()))
        return pf, ps

    def save(self, path):
        _check(lib().rt_unet_save(self.h, os.fsencode(path)))

    def load(self, path):
        _check(lib().rt_unet_load(self.h, os.fsencode(path)))


def rt_segment_tile_surrogate(rgb, net, tau=0.5, params=None, ctx=None):
    """Returns (mask, labels, n_objects, used_fallback, confidence)."""
    ctx = ctx or net.ctx
    _img(rgb, torch.uint8, "rgb", 3)
    h, w = rgb.shape[:2]
    p = params if params is not None else default_params()
    mask = torch.empty((h, w), dtype=torch.uint8, device=rgb.device)
    lab = torch.empty((h, w), dtype=torch.int32, device=rgb.device)
    n = torch.zeros(1, dtype=torch.int32, device=rgb.device)
    fb = C.c_int32(0)
    conf = C.c_float(0.0)
    _check(lib().rt_segment_tile_surrogate(ctx.h, net.h, _ptr(rgb), rgb.stride(0), w, h, C.byref(p), float(tau),
                                           _ptr(mask), _ptr(lab), w, _ptr(n), C.byref(fb), C.byref(conf),
                                           _stream()))
    return mask, lab, n, bool(fb.value), float(conf.value)


def _u16(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype not in (torch.int16, torch.uint16, torch.bfloat16):
        raise TypeError(f"{name}: expected a 16-bit device tensor holding bfloat16")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    return t


def nn_conv3_fwd(x0, wf, bias, co, relu=False, x1=None, want_bf16=False, ctx=None):
    """x0 (n, h, w, c0) [and x1 (n, h, w, c1)] bf16 -> y float32 (n, h, w, co)
    [and, with want_bf16, the same output rounded to bf16 by the kernel]."""
    ctx = ctx or default_context()
    n, h, w, c0 = x0.shape
    c1 = x1.shape[3] if x1 is not None else 0
    y = torch.empty((n, h, w, co), dtype=torch.float32, device=x0.device)
    yb = torch.empty((n, h, w, co), dtype=torch.int16, device=x0.device) if want_bf16 else None
    _check(lib().rt_nn_conv3_fwd(ctx.h, _ptr(_u16(x0, "x0")), c0, _ptr(x1), c1, n, h, w, _ptr(_u16(wf, "wf")),
                                 _ptr(bias), co, 1 if relu else 0, _ptr(y), _ptr(yb), _stream()))
    return (y, yb) if want_bf16 else y


def nn_conv3_dgrad(g, wt, ci, c0=None, ctx=None):
    ctx = ctx or default_context()
    n, h, w, co = g.shape
    c0 = ci if c0 is None else c0
    dx0 = torch.empty((n, h, w, c0), dtype=torch.float32, device=g.device)
    dx1 = torch.empty((n, h, w, ci - c0), dtype=torch.float32, device=g.device) if c0 < ci else None
    _check(lib().rt_nn_conv3_dgrad(ctx.h, _ptr(_u16(g, "g")), co, n, h, w, _ptr(_u16(wt, "wt")), ci, c0, _ptr(dx0),
                                   _ptr(dx1), _stream()))
    return (dx0, dx1) if dx1 is not None else dx0


def nn_conv3_wgrad(x0, g, x1=None, ctx=None):
    ctx = ctx or default_context()
    n, h, w, c0 = x0.shape
    c1 = x1.shape[3] if x1 is not None else 0
    co = g.shape[3]
    dw = torch.zeros((co, 9, c0 + c1), dtype=torch.float32, device=x0.device)
    db = torch.zeros(co, dtype=torch.float32, device=x0.device)
    _check(lib().rt_nn_conv3_wgrad(ctx.h, _ptr(_u16(x0, "x0")), c0, _ptr(x1), c1, _ptr(_u16(g, "g")), co, n, h, w,
                                   _ptr(dw), _ptr(db), _stream()))
    return dw, db


def nn_up2_fwd(x, uf, bias, co, want_bf16=False, ctx=None):
    ctx = ctx or default_context()
    n, h, w, ci = x.shape
    y = torch.empty((n, 2 * h, 2 * w, co), dtype=torch.float32, device=x.device)
    yb = torch.empty((n, 2 * h, 2 * w, co), dtype=torch.int16, device=x.device) if want_bf16 else None
    _check(lib().rt_nn_up2_fwd(ctx.h, _ptr(_u16(x, "x")), ci, n, h, w, _ptr(_u16(uf, "uf")), _ptr(bias), co, _ptr(y),
                               _ptr(yb), _stream()))
    return (y, yb) if want_bf16 else y


def nn_up2_bwd(x, g, ut, ctx=None):
    ctx = ctx or default_context()
    n, h, w, ci = x.shape
    co = g.shape[3]
    dx = torch.empty((n, h, w, ci), dtype=torch.float32, device=x.device)
    dw = torch.zeros((ci, 4, co), dtype=torch.float32, device=x.device)
    db = torch.zeros(co, dtype=torch.float32, device=x.device)
    _check(lib().rt_nn_up2_bwd(ctx.h, _ptr(_u16(x, "x")), ci, _ptr(_u16(g, "g")), co, n, h, w, _ptr(_u16(ut, "ut")),
                               _ptr(dx), _ptr(dw), _ptr(db), _stream()))
    return dx, dw, db


def nn_pool2_fwd(x, ctx=None):
    ctx = ctx or default_context()
    n, h, w, c = x.shape
    y = torch.empty((n, h // 2, w // 2, c), dtype=x.dtype, device=x.device)
    idx = torch.empty((n, h // 2, w // 2, c), dtype=torch.uint8, device=x.device)
    _check(lib().rt_nn_pool2(ctx.h, _ptr(_u16(x, "x")), c, n, h, w, _ptr(y), _ptr(idx), None, None, _stream()))
    return y, idx


def nn_pool2_bwd(dy, idx, dx, ctx=None):
    """dx (n, h, w, c) float32 += unpool(dy)."""
    ctx = ctx or default_context()
    n, h, w, c = dx.shape
    _check(lib().rt_nn_pool2(ctx.h, None, c, n, h, w, None, _ptr(idx), _ptr(dy), _ptr(dx), _stream()))
    return dx


def nn_head_loss(x, wh, bh, t_fg, t_seed, w_seed=1.0, ctx=None):
    """Returns (loss, dx, dw, db) of the 1x1 head + loss on x (n, h, w, 16) bf16."""
    ctx = ctx or default_context()
    n, h, w, _ = x.shape
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    dx = torch.empty((n, h, w, 16), dtype=torch.float32, device=x.device)
    dw = torch.zeros((2, 16), dtype=torch.float32, device=x.device)
    db = torch.zeros(2, dtype=torch.float32, device=x.device)
    _check(lib().rt_nn_head_loss(ctx.h, _ptr(_u16(x, "x")), n, h, w, _ptr(wh), _ptr(bh), _ptr(t_fg), _ptr(t_seed),
                                 float(w_seed), _ptr(loss), _ptr(dx), _ptr(dw), _ptr(db), _stream()))
    return loss, dx, dw, db


def nn_pack(kind, w, ci, co, ctx=None):
    """bfloat16 operand copies (fwd, tr) of a float32 weight: kind 0 conv3
    [co][9][ci], kind 1 up2 [ci][4][co]."""
    ctx = ctx or default_context()
    fwd = torch.empty(w.numel(), dtype=torch.int16, device=w.device)
    tr = torch.empty(w.numel(), dtype=torch.int16, device=w.device)
    _check(lib().rt_nn_pack(ctx.h, int(kind), _ptr(w), ci, co, _ptr(fwd), _ptr(tr), _stream()))
    return fwd, tr


def nn_prep_input(rgb, ctx=None):
    ctx = ctx or default_context()
    _img(rgb, torch.uint8, "rgb", 3)
    h, w = rgb.shape[:2]
    x = torch.empty((1, h, w, 8), dtype=torch.int16, device=rgb.device)
    _check(lib().rt_nn_prep_input(ctx.h, _ptr(rgb), rgb.stride(0), w, h, _ptr(x), _stream()))
    return x


EXPORTS = ("rt_ctx_create", "rt_ctx_destroy", "rt_last_error", "rt_sync", "rt_deconv", "rt_morph_recon",
           "rt_fill_holes", "rt_ccl", "rt_ccl_noalloc", "rt_features", "rt_morph", "rt_recon_to_nuclei", "rt_rbc_detect", "rt_area_filter", "rt_watershed", "rt_seg_params_default",
           "rt_segment_tile", "rt_segment_batch", "rt_segment_host_stream", "rt_segment_slide", "rt_set_knob", "rt_get_knob", "rt_profile_enable", "rt_profile_read", "rt_profile_recon_rounds", "rt_profile_objects",
           "rt_profile_stage_name", "rt_unet_param_count", "rt_unet_create", "rt_unet_destroy", "rt_unet_get_params",
           "rt_unet_set_params", "rt_unet_get_grads", "rt_unet_grad_step", "rt_unet_train_step", "rt_unet_forward",
           "rt_unet_save", "rt_unet_load", "rt_unet_adam_step", "rt_unet_get_step", "rt_unet_save_checkpoint",
           "rt_unet_load_checkpoint", "rt_segment_tile_surrogate", "rt_nn_conv3_fwd", "rt_nn_conv3_dgrad",
           "rt_nn_conv3_wgrad", "rt_nn_up2_fwd", "rt_nn_up2_bwd", "rt_nn_pool2", "rt_nn_head_loss", "rt_nn_pack",
           "rt_nn_prep_input")
