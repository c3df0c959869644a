"""Pins of the pre-processing oracle (oracle/morph_oracle.c) on the CPU:
erosion and dilation by the flat disk against scipy.ndimage (outside pixels
ignored), opening as their composition and its algebraic properties, the
ReconToNuclei markers (frame marker against the whole-pipeline oracle,
opening by reconstruction against iterated geodesic dilation and its
bounds), and RBC detection against a scipy labelling of the hysteresis
definition."""
import numpy as np
import pytest
from scipy import ndimage

from tests import brute


def disk(r):
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    return (xx * xx + yy * yy) <= r * r


@pytest.mark.parametrize("r", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("seed", [0, 1])
def test_erode_dilate_against_scipy(oracle, r, seed):
    rng = np.random.Generator(np.random.PCG64(40 + seed))
    img = rng.integers(0, 256, size=(int(rng.integers(8, 40)), int(rng.integers(8, 40))), dtype=np.uint8)
    fp = disk(r)
    # outside pixels never win: pad with the neutral value of each operator
    e = ndimage.grey_erosion(img, footprint=fp, mode="constant", cval=255)
    d = ndimage.grey_dilation(img, footprint=fp, mode="constant", cval=0)
    assert np.array_equal(oracle.erode(img, r), e)
    assert np.array_equal(oracle.dilate(img, r), d)
    assert np.array_equal(oracle.open_(img, r), ndimage.grey_dilation(e, footprint=fp, mode="constant", cval=0))


def test_disk_shape_by_hand(oracle):
    img = np.zeros((9, 9), np.uint8)
    img[4, 4] = 200
    d = oracle.dilate(img, 2)
    assert d.sum() == 200 * 13   # the radius-2 disk holds 13 pixels: 1 + 4 + 4 + 4
    assert d[4, 2] == 200 and d[2, 4] == 200 and d[3, 3] == 200 and d[2, 3] == 0


@pytest.mark.parametrize("r", [1, 3])
def test_opening_properties(oracle, r):
    rng = np.random.Generator(np.random.PCG64(77 + r))
    img = ndimage.uniform_filter(rng.integers(0, 256, size=(48, 52)).astype(float), 3).astype(np.uint8)
    o = oracle.open_(img, r)
    assert (o <= img).all()                                    # anti-extensive
    assert np.array_equal(oracle.open_(o, r), o)               # idempotent
    brighter = np.minimum(img.astype(int) + 10, 255).astype(np.uint8)
    assert (oracle.open_(brighter, r) >= o).all()              # increasing


def test_frame_marker_matches_the_pipeline(oracle):
    from paper_1405_7958_amd import synth
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    hq = oracle.deconv(rgb)
    r, f0 = oracle.recon_to_nuclei(hq, oracle.MARKER_FRAME, 0, 16)
    _, _, _, inter = oracle.segment_from_hq(hq, intermediates=True)
    assert np.array_equal(r, inter["R"]) and np.array_equal(f0, inter["F0"])


@pytest.mark.parametrize("seed", range(4))
def test_opening_by_reconstruction_marker(oracle, seed):
    rng = np.random.Generator(np.random.PCG64(300 + seed))
    h, w = int(rng.integers(10, 24)), int(rng.integers(10, 24))
    hq = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    r = int(rng.integers(1, 4))
    R, f0 = oracle.recon_to_nuclei(hq, oracle.MARKER_OPEN, r, 16)
    ero = oracle.erode(hq, r)
    exp = brute.recon_iterate(ero.astype(np.int64), hq.astype(np.int64), None, 8)
    assert np.array_equal(R, exp)
    assert (R >= oracle.open_(hq, r)).all() and (R <= hq).all() and (R >= ero).all()
    assert np.array_equal(f0, ((hq.astype(int) - R) >= 16).astype(np.uint8))


def test_rbc_detection_hysteresis(oracle):
    rng = np.random.Generator(np.random.PCG64(5))
    h, w = 60, 70
    rgb = np.empty((h, w, 3), np.uint8)
    rgb[...] = (230, 180, 200)
    yy, xx = np.mgrid[0:h, 0:w]
    for cy, cx, rr, col in [(15, 15, 6, (215, 60, 70)), (40, 50, 5, (190, 120, 110)), (45, 15, 4, (120, 70, 150))]:
        rgb[(yy - cy) ** 2 + (xx - cx) ** 2 <= rr * rr] = col
    rgb = np.clip(rgb.astype(int) + rng.integers(-6, 7, size=rgb.shape), 0, 255).astype(np.uint8)
    t_s, t_w = 200, 150
    red = 2 * rgb[..., 0].astype(int) - rgb[..., 1] - rgb[..., 2]
    lab, n = ndimage.label(red >= t_w, structure=np.ones((3, 3)))
    keep = np.unique(lab[(red >= t_s) & (lab > 0)])
    exp = np.isin(lab, keep[keep > 0]).astype(np.uint8)
    got = oracle.rbc_detect(rgb, t_s, t_w)
    assert np.array_equal(got, exp)
    # the bright red disc is found whole, the pale one (redness ~150-170, no
    # strong pixel) and the nucleus are not
    assert got[15, 15] == 1 and got[40, 50] == 0 and got[45, 15] == 0
