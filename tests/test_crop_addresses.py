"""Host-side bounds check of the per-object kernels' crop loads: the loads
are issued in batches with addresses clamped into each component's crop
(paper_1405_7958_amd/csrc/crop_addr.h); tests/crop_addr_check.cpp walks
every load of every component through that same address function and
checks that it addresses a pixel of the crop.  The components are those of
the GPU tests' own inputs (the external-seeds watershed input, the
every-class watershed input, the segmented 512 x 512 tile) plus boxes on
every edge and corner of the image, one-pixel-wide boxes and the whole
image, with dense and padded pitches."""
import os
import subprocess

import numpy as np
import pytest
from scipy import ndimage

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("crop") / "crop_addr_check")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O2", "-x", "hip",
                           os.path.join(ROOT, "tests", "crop_addr_check.cpp"),
                           "-I", os.path.join(ROOT, "paper_1405_7958_amd", "csrc"), "-o", exe])
    return exe


def run(checker, w, h, pitch, boxes):
    text = f"{w} {h} {pitch} {len(boxes)}\n" + "".join(f"{a} {b} {c} {d}\n" for a, b, c, d in boxes)
    r = subprocess.run([checker], input=text, capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
    return int(r.stdout.split()[1])


def boxes_of(fg):
    lab, _ = ndimage.label(fg, structure=np.ones((3, 3)))
    out = []
    for sl in ndimage.find_objects(lab):
        if sl is not None:
            out.append((sl[1].start, sl[0].start, sl[1].stop - 1, sl[0].stop - 1))
    return out


def blobs(h, w, n, seed, rmin=3, rmax=12):
    # the generator of the GPU watershed tests
    r = np.random.Generator(np.random.PCG64(seed))
    yy, xx = np.mgrid[0:h, 0:w]
    fg = np.zeros((h, w), bool)
    for _ in range(n):
        cy, cx = r.uniform(0, h), r.uniform(0, w)
        a, b = r.uniform(rmin, rmax), r.uniform(rmin, rmax)
        t = r.uniform(0, np.pi)
        u = ((xx - cx) * np.cos(t) + (yy - cy) * np.sin(t)) / a
        v = (-(xx - cx) * np.sin(t) + (yy - cy) * np.cos(t)) / b
        fg |= u * u + v * v <= 1
    return fg


@pytest.mark.parametrize("pad", [0, 7, 64])
def test_watershed_inputs(checker, pad):
    fg = blobs(256, 256, 120, seed=9)     # the external-seeds watershed input
    assert run(checker, 256, 256, 256 + pad, boxes_of(fg)) > 0
    for h, w, n in [(64, 64, 12), (200, 300, 60), (333, 517, 150)]:
        fg = blobs(h, w, n, seed=h + w)
        run(checker, w, h, w + pad, boxes_of(fg))


def test_segmented_512_components(checker, oracle):
    from paper_1405_7958_amd import synth
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    _, _, _, inter = oracle.segment_from_hq(oracle.deconv(rgb), intermediates=True)
    run(checker, 512, 512, 512, boxes_of(inter["F"]))


@pytest.mark.parametrize("w,h", [(1, 1), (1, 90), (90, 1), (33, 33), (65, 64), (256, 256)])
def test_edge_boxes(checker, w, h):
    boxes = [(0, 0, w - 1, h - 1), (0, 0, 0, 0), (w - 1, h - 1, w - 1, h - 1), (w - 1, 0, w - 1, h - 1),
             (0, h - 1, w - 1, h - 1), (0, 0, min(w, 31) - 1, min(h, 31) - 1),
             (max(0, w - 31), max(0, h - 31), w - 1, h - 1), (max(0, w - 63), 0, w - 1, min(h, 62) - 1)]
    for pad in (0, 1, 3):
        run(checker, w, h, w + pad, boxes)
