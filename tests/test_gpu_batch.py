"""Batched segmentation (rt_segment_batch) against the CPU oracle.

Every tile of a batch must give exactly what the oracle gives for that tile
alone: Hq within 1 LSB of the FP64 oracle, then mask, labels and object count
bit-exact with the oracle re-run from the GPU's own Hq.  The oracle runs on
host threads (its C entry points release the GIL), one tile per thread.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests.gpu_util import assert_equal, dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()   # fails loudly if the HIP library is missing
    return rtseg


def _gen(specs):
    with ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(lambda s: synth.make_tile(s)[0], specs))


def _check_batch(rt, oracle, rgbs, what, hq_check=None):
    d = dev()
    say("segment_batch", what, len(rgbs), "tiles")
    outs = rt.rt_segment_batch([to_dev(r, d) for r in rgbs], want_hq=True)
    got = [tuple(to_np(t) for t in o) for o in outs]
    hq_check = range(len(rgbs)) if hq_check is None else hq_check

    def expect(i):
        ohq = oracle.deconv(rgbs[i]) if i in hq_check else None
        return ohq, oracle.segment_from_hq(got[i][3])

    with ThreadPoolExecutor(WORKERS) as ex:
        exp = list(ex.map(expect, range(len(rgbs))))
    total = 0
    for i, ((mask, lab, n, hq), (ohq, (emask, elab, en))) in enumerate(zip(got, exp)):
        if ohq is not None:
            assert np.abs(hq.astype(int) - ohq.astype(int)).max() <= 1, f"{what} tile {i} Hq"
        assert_equal(mask, emask, f"{what} tile {i} {rgbs[i].shape} mask")
        assert_equal(lab, elab, f"{what} tile {i} {rgbs[i].shape} labels")
        assert int(n[0]) == en, (what, i, int(n[0]), en)
        total += en
    return total


def test_batch_uneven_64(rt, oracle):
    """The 64-tile batch of uneven slide-edge sizes (512..4096 per side,
    300-800 nuclei per Mpx), every tile compared whole."""
    specs = [synth.spec_uneven(i) for i in range(64)]
    rgbs = _gen(specs)
    # the FP64 deconvolution oracle is checked on every tile up to 2048 x 2048
    small = {i for i, s in enumerate(specs) if s.w * s.h <= 2048 * 2048}
    n = _check_batch(rt, oracle, rgbs, "uneven64", hq_check=small)
    assert n > 1000


def test_batch_ragged_and_degenerate(rt, oracle):
    rng = np.random.Generator(np.random.PCG64(77))
    rgbs = [np.full((96, 80, 3), 255, np.uint8),
            np.tile(np.array([120, 70, 150], np.uint8), (33, 65, 1)),
            synth.random_rgb(1, 1, seed=1), synth.random_rgb(1, 64, seed=2), synth.random_rgb(37, 1, seed=3)]
    for k in range(11):
        h, w = (int(v) for v in rng.integers(1, 700, size=2))
        spec = synth.TileSpec(w=w, h=h, seed=100 + k, n_nuclei=max(1, w * h // 2500), amin=4, amax=14,
                              cluster_frac=0.3, cluster_min=2, cluster_max=4, jitter=20)
        rgbs.append(synth.make_tile(spec)[0])
    _check_batch(rt, oracle, rgbs, "ragged")


def test_batch_several_launch_groups(rt, oracle):
    """More tiles than one launch group holds (64), mixed with dense tiles."""
    specs = []
    for i in range(150):
        s = synth.spec_stream(i)
        w, h = 64 + (s.w % 300), 48 + (s.h % 260)
        specs.append(synth.TileSpec(w=w, h=h, seed=s.seed, n_nuclei=max(1, int(s.n_nuclei * w * h / (s.w * s.h))),
                                    amin=4, amax=14, cluster_frac=s.cluster_frac, cluster_min=s.cluster_min,
                                    cluster_max=s.cluster_max, jitter=s.jitter, low_contrast=s.low_contrast))
    _check_batch(rt, oracle, _gen(specs), "groups")


def test_batch_matches_single_tile_calls(rt):
    d = dev()
    rgbs = [synth.make_tile(synth.spec_uneven(i))[0] for i in (3, 5)]
    rgbs.append(synth.make_tile(synth.spec_small(1))[0])
    say("segment_batch vs single")
    outs = rt.rt_segment_batch([to_dev(r, d) for r in rgbs])
    for i, r in enumerate(rgbs):
        m, l, n = rt.rt_segment_tile(to_dev(r, d))
        assert_equal(to_np(outs[i][1]), to_np(l), f"tile {i} labels")
        assert_equal(to_np(outs[i][0]), to_np(m), f"tile {i} mask")
        assert int(to_np(outs[i][2])[0]) == int(to_np(n)[0])


def test_batch_empty_and_bad_arguments(rt):
    import ctypes as C
    import torch
    d = dev()
    assert rt.rt_segment_batch([]) == []
    ctx = rt.default_context(0)
    p = rt.default_params()
    rgb = torch.zeros((8, 8, 3), dtype=torch.uint8, device=d)
    m = torch.zeros((8, 8), dtype=torch.uint8, device=d)
    lab = torch.zeros((8, 8), dtype=torch.int32, device=d)
    bad = [rt.rt_tile_desc(rgb.data_ptr(), 24, 8, 8, m.data_ptr(), lab.data_ptr(), 8, None, None),
           rt.rt_tile_desc(rgb.data_ptr(), 24, 0, 8, m.data_ptr(), lab.data_ptr(), 8, None, None)]
    arr = (rt.rt_tile_desc * 2)(*bad)
    rc = rt.lib().rt_segment_batch(ctx.h, 2, arr, C.byref(p), None)
    assert rc == rt.RT_EINVAL and b"tile 1" in rt.lib().rt_last_error()
    big = rt.rt_tile_desc(rgb.data_ptr(), 3 * 6000, 6000, 6000, m.data_ptr(), lab.data_ptr(), 6000, None, None)
    rc = rt.lib().rt_segment_batch(ctx.h, 1, (rt.rt_tile_desc * 1)(big), C.byref(p), None)
    assert rc == rt.RT_EINVAL
