"""Host-resident tile streams (rt_segment_host_stream): tiles in host memory,
uploads / computation / downloads overlapped on three streams.  Every result
must equal rt_segment_tile's on the same tile (bit-exact masks, labels and
counts), for every pipeline depth, with uneven tile sizes (so the device
slots are reused by tiles of other sizes), pinned and pageable host memory,
outputs left out, and an empty list; one tile is also checked against the
oracle re-run from the GPU's Hq."""
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


@pytest.fixture(scope="module")
def tiles():
    import torch
    out = []
    for i, (w, h) in enumerate([(512, 512), (1024, 512), (300, 700), (512, 512), (777, 333)]):
        spec = synth.TileSpec(w=w, h=h, seed=40000 + i, n_nuclei=int(600 * w * h / 1e6), amin=4, amax=14,
                              cluster_frac=0.2, cluster_min=2, cluster_max=4, jitter=20)
        out.append(torch.from_numpy(synth.make_tile(spec)[0]))
    return out


def _reference(rt, tiles, d):
    ref = []
    for t in tiles:
        m, lab, n, hq = rt.rt_segment_tile(to_dev(t.numpy(), d), want_hq=True)
        ref.append((to_np(m), to_np(lab), int(to_np(n)[0]), to_np(hq)))
    return ref


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_host_stream_matches_device_calls(rt, tiles, depth):
    d = dev()
    ref = _reference(rt, tiles, d)
    pinned = [t.pin_memory() for t in tiles]
    say("host stream depth", depth)
    got = rt.rt_segment_host_stream(pinned, depth=depth)
    for i, ((m, lab, cnt), (em, elab, en, _)) in enumerate(zip(got, ref)):
        assert_equal(m.numpy(), em, f"depth {depth} tile {i} mask")
        assert_equal(lab.numpy(), elab, f"depth {depth} tile {i} labels")
        assert int(cnt[0]) == en


def test_host_stream_against_oracle_pageable_and_partial(rt, oracle, tiles):
    d = dev()
    ref = _reference(rt, tiles[:2], d)
    say("host stream pageable, labels only")
    got = rt.rt_segment_host_stream(tiles[:2], depth=3, want_mask=False)
    for i, ((m, lab, cnt), (em, elab, en, hq)) in enumerate(zip(got, ref)):
        assert m is None
        assert_equal(lab.numpy(), elab, f"pageable tile {i} labels")
        emask, olab, on = oracle.segment_from_hq(hq)
        assert_equal(lab.numpy(), olab, f"pageable tile {i} labels vs oracle")
        assert int(cnt[0]) == en == on
    say("host stream empty")
    assert rt.rt_segment_host_stream([], depth=3) == []
    with pytest.raises(rt.RtError):
        rt.rt_segment_host_stream(tiles[:1], depth=4)
