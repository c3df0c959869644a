"""The work-queue reconstruction against the oracle, alone (recon_mode 1) and
after a round of launches (recon_mode 2): single reconstructions (u8 /
int32, 4 / 8 connectivity, domains, a spiral whose path crosses every tile),
whole tiles, and graph replays of a batch."""
import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests.gpu_util import assert_equal, dev, say, to_dev, to_np
from tests.test_gpu_parity import _recon_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()
    return rtseg


@pytest.fixture(scope="module", params=[1, 2])
def qctx(rt, request):
    c = rt.Context(0)
    rt.rt_set_knob("recon_mode", request.param, ctx=c)
    rt.rt_set_knob("recon_queue_after", 1, ctx=c)
    yield c
    c.close()


@pytest.mark.parametrize("dtype", [np.uint8, np.int32])
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape,dom", [((1, 1), False), ((37, 200), True), ((300, 301), False)])
def test_queue_recon_random(rt, oracle, qctx, dtype, conn, shape, dom):
    d = dev()
    J, I, D = _recon_case(shape[0] * 7 + shape[1], shape[0], shape[1], dtype, dom)
    say("queue recon", dtype.__name__, conn, shape, dom)
    got = rt.rt_morph_recon(to_dev(J, d), to_dev(I, d), to_dev(D, d) if D is not None else None, conn, ctx=qctx)
    assert_equal(to_np(got), oracle.recon(J, I, D, conn).astype(dtype), f"queue recon {shape}")


def test_queue_recon_spiral(rt, oracle, qctx):
    d = dev()
    s = (synth.spiral(300, 280) * 200).astype(np.uint8)
    J = np.zeros_like(s)
    J[0, 0] = 200
    for conn in (4, 8):
        say("queue spiral", conn)
        got = rt.rt_morph_recon(to_dev(J, d), to_dev(s, d), None, conn, ctx=qctx)
        assert_equal(to_np(got), oracle.recon(J, s, None, conn).astype(np.uint8), f"queue spiral conn={conn}")


@pytest.mark.parametrize("levels", [0, 3])
def test_queue_segment_tiles(rt, oracle, qctx, levels):
    d = dev()
    rt.rt_set_knob("recon_levels", levels, ctx=qctx)
    for name, spec in [("small", synth.spec_small(5)), ("4k", synth.spec_4k(0))]:
        rgb = synth.make_tile(spec)[0]
        say("queue segment", name, levels)
        mask, lab, n, hq = rt.rt_segment_tile(to_dev(rgb, d), want_hq=True, ctx=qctx)
        emask, elab, en = oracle.segment_from_hq(to_np(hq))
        assert_equal(to_np(lab), elab, f"queue {name} labels")
        assert_equal(to_np(mask), emask, f"queue {name} mask")
        assert int(to_np(n)[0]) == en
    rt.rt_set_knob("recon_levels", 3, ctx=qctx)


@pytest.mark.parametrize("mode", [1, 2])
def test_queue_batch_graph_replays(rt, oracle, mode):
    import torch
    d = dev()
    c = rt.Context(0)
    rt.rt_set_knob("recon_mode", mode, ctx=c)
    specs = [synth.spec_uneven(i) for i in (0, 2)]
    specs = [synth.TileSpec(w=min(s.w, 1024), h=min(s.h, 1024), seed=s.seed, n_nuclei=s.n_nuclei // 4, amin=4,
                            amax=14, cluster_frac=0.2, cluster_min=2, cluster_max=4, jitter=20) for s in specs]
    rgbs = [to_dev(synth.make_tile(s)[0], d) for s in specs]
    say("queue batch eager")
    ref = [tuple(to_np(x) for x in o) for o in rt.rt_segment_batch(rgbs, want_hq=True, ctx=c)]
    for i, r in enumerate(ref):
        emask, elab, en = oracle.segment_from_hq(r[3])
        assert_equal(r[1], elab, f"queue batch tile {i}")
    rt.rt_set_knob("graph", 1, ctx=c)
    for rep in range(3):
        say("queue batch graph", rep)
        got = rt.rt_segment_batch(rgbs, ctx=c)
        torch.cuda.synchronize()
        for i, (g, r) in enumerate(zip(got, ref)):
            assert_equal(to_np(g[1]), r[1], f"queue graph replay {rep} tile {i}")
    c.close()
