"""Pre-processing entry points against the CPU oracle, through the C ABI,
bit-exact: flat-disk erosion, dilation and opening (radii 0 to the maximum,
sizes spanning several 64 x 32 tiles with ragged edges, one-pixel-wide
images, a pitched input, the 4096 x 4096 Hq); ReconToNuclei with the frame
and the opening-by-reconstruction marker; RBC detection."""
import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests.gpu_util import assert_equal, dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()   # fails loudly if the HIP library is missing
    return rtseg


ORACLE_OP = {0: "erode", 1: "dilate", 2: "open_"}


@pytest.mark.parametrize("h,w,r", [(100, 150, 0), (100, 150, 1), (333, 517, 3), (65, 33, 7), (1, 70, 2),
                                   (70, 1, 2), (97, 129, 32)])
def test_morph_ops(rt, oracle, h, w, r):
    d = dev()
    rng = np.random.Generator(np.random.PCG64(h * 1000 + w + r))
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    for op in (0, 1, 2):
        say("morph", ORACLE_OP[op], h, w, r)
        got = to_np(rt.rt_morph(to_dev(img, d), op, r))
        assert_equal(got, getattr(oracle, ORACLE_OP[op])(img, r), f"{ORACLE_OP[op]} {h}x{w} r={r}")


def test_morph_pitched_and_rejects(rt, oracle):
    import torch
    d = dev()
    rng = np.random.Generator(np.random.PCG64(61))
    img = rng.integers(0, 256, size=(90, 120), dtype=np.uint8)
    big = torch.zeros((90, 160), dtype=torch.uint8, device=d)
    big[:, :120] = to_dev(img, d)
    say("morph pitched")
    assert_equal(to_np(rt.rt_morph(big[:, :120], 2, 4)), oracle.open_(img, 4), "open pitched")
    with pytest.raises(rt.RtError):
        rt.rt_morph(big[:, :120], 0, 33)


def test_morph_open_4k_hq(rt, oracle):
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_4k(0))
    say("morph open on the 4096 Hq")
    hq = rt.rt_deconv(to_dev(rgb, d))
    assert_equal(to_np(rt.rt_morph(hq, 2, 5)), oracle.open_(to_np(hq), 5), "open 4096 r=5")


@pytest.mark.parametrize("marker,radius", [(0, 0), (1, 3), (1, 6)])
def test_recon_to_nuclei_markers(rt, oracle, marker, radius):
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    hq = rt.rt_deconv(to_dev(rgb, d))
    say("recon_to_nuclei", marker, radius)
    R, f0 = rt.rt_recon_to_nuclei(hq, marker, radius, 16)
    eR, ef0 = oracle.recon_to_nuclei(to_np(hq), marker, radius, 16)
    assert_equal(to_np(R), eR, f"R marker={marker} r={radius}")
    assert_equal(to_np(f0), ef0, f"F0 marker={marker} r={radius}")


def _rbc_tile(h, w, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rgb = np.empty((h, w, 3), np.float64)
    rgb[...] = (230, 180, 200)
    yy, xx = np.mgrid[0:h, 0:w]
    for _ in range(n):
        cy, cx, rr = rng.integers(0, h), rng.integers(0, w), rng.uniform(3, 9)
        col = [(215, 60, 70), (190, 120, 110), (120, 70, 150)][int(rng.integers(0, 3))]
        rgb[(yy - cy) ** 2 + (xx - cx) ** 2 <= rr * rr] = col
    return np.clip(np.rint(rgb + rng.normal(0, 8, size=rgb.shape)), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("h,w,seed", [(300, 400, 1), (129, 700, 2)])
def test_rbc_detect(rt, oracle, h, w, seed):
    d = dev()
    rgb = _rbc_tile(h, w, h * w // 1500, 700 + seed)
    say("rbc", h, w)
    got = to_np(rt.rt_rbc_detect(to_dev(rgb, d), 200, 150))
    exp = oracle.rbc_detect(rgb, 200, 150)
    assert_equal(got, exp, f"rbc {h}x{w}")
    assert exp.sum() > 0
