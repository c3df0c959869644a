"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["rt_deconv", "rt_morph_recon", "rt_fill_holes", "rt_ccl", "rt_area_filter", "rt_watershed",
              "rt_segment_tile", "rt_segment_batch"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1405_7958_amd import rtseg
    if not os.path.exists(rtseg.LIB_PATH):
        pytest.fail("librtseg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(rtseg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_the_boundary():
    from paper_1405_7958_amd import rtseg
    for n in ["rt_deconv", "rt_morph_recon", "rt_fill_holes", "rt_ccl", "rt_area_filter", "rt_watershed",
              "rt_segment_tile", "rt_segment_batch"]:
        assert callable(getattr(rtseg, n))


def test_params_struct_layout_matches_header():
    from paper_1405_7958_amd import rtseg
    # uint32 size; 9 doubles; 1 double; 5 int32 (with alignment padding after size)
    assert ctypes.sizeof(rtseg.rt_seg_params) == 8 + 9 * 8 + 8 + 5 * 4 + 4


def test_tile_desc_struct_layout_matches_header():
    from paper_1405_7958_amd import rtseg
    # ptr, int64, 2 x int32, ptr, ptr, int64, ptr, ptr, ptr, ptr
    assert ctypes.sizeof(rtseg.rt_tile_desc) == 8 + 8 + 4 + 4 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert rtseg.rt_tile_desc.w.offset == 16 and rtseg.rt_tile_desc.mask_out.offset == 24


def test_binding_exports_list_matches_headers():
    from paper_1405_7958_amd import rtseg
    assert set(_declared()) == set(rtseg.EXPORTS)
