"""Cross-tile stitching (rt_segment_slide) against the stitching oracle re-run
from the GPU's slide Hq, bit-exact: ragged cores, a halo, no halo, one core
covering the slide, more cores than one launch group holds, and the
asynchronous reconstruction mode."""
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


def slide(w, h, seed):
    spec = synth.TileSpec(w=w, h=h, seed=seed, n_nuclei=int(700 * w * h / 1e6), amin=4, amax=14,
                          cluster_frac=0.2, cluster_min=2, cluster_max=4, jitter=20)
    return synth.make_tile(spec)[0]


@pytest.mark.parametrize("w,h,tile,halo", [(520, 390, 96, 40), (520, 390, 128, 0), (300, 200, 512, 32),
                                           (1000, 900, 100, 24)])
def test_stitch_matches_oracle(rt, oracle, w, h, tile, halo):
    d = dev()
    rgb = to_dev(slide(w, h, 62000 + w + tile), d)
    say("stitch", w, h, tile, halo)
    lab, mask, n, hq = rt.rt_segment_slide(rgb, tile, halo, want_hq=True)
    elab, emask, en = oracle.stitch_from_hq(to_np(hq), tile, halo)
    assert_equal(to_np(lab), elab, f"stitch {w}x{h} tile {tile} halo {halo} labels")
    assert_equal(to_np(mask), emask, f"stitch {w}x{h} tile {tile} halo {halo} mask")
    assert int(to_np(n)[0]) == en
    ohq = oracle.deconv(to_np(rgb))
    assert np.abs(ohq.astype(int) - to_np(hq).astype(int)).max() <= 1


def test_stitch_one_core_and_async(rt, oracle):
    d = dev()
    rgb = to_dev(slide(700, 500, 62900), d)
    say("stitch one core")
    lab, mask, n = rt.rt_segment_slide(rgb, 1024, 16)
    m2, l2, n2 = rt.rt_segment_tile(rgb)
    assert_equal(to_np(lab), to_np(l2), "one core vs rt_segment_tile")
    assert int(to_np(n)[0]) == int(to_np(n2)[0])
    ctx = rt.Context(0)
    rt.rt_set_knob("recon_async", 1, ctx=ctx)
    say("stitch async")
    la, ma, na, hqa = rt.rt_segment_slide(rgb, 160, 40, want_hq=True, ctx=ctx)
    elab, emask, en = oracle.stitch_from_hq(to_np(hqa), 160, 40)
    assert_equal(to_np(la), elab, "stitch async labels")
    assert int(to_np(na)[0]) == en
    ctx.close()
