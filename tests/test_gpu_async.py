"""Asynchronous segmentation (knob recon_async): the reconstruction rounds
run to convergence without the host reading the worklist -- launched rounds,
then a one-workgroup finish on the device.  Results must equal the oracle's
(re-run from the GPU's Hq) and the synchronous mode's, bit-exact, also when
only one round is launched (the device finish does nearly all the work), for
batches of uneven tiles, and for graph replays; the host reads no worklist
counter in this mode."""
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


def _ctx(rt, **knobs):
    ctx = rt.Context(0)
    for k, v in knobs.items():
        rt.rt_set_knob(k, v, ctx=ctx)
    return ctx


@pytest.mark.parametrize("rounds", [16, 3, 1])
def test_async_single_tile_matches_oracle(rt, oracle, rounds):
    d = dev()
    rgb = to_dev(synth.make_tile(synth.spec_small(0))[0], d)
    ctx = _ctx(rt, recon_async=1, recon_async_rounds=rounds)
    reads0 = rt.rt_get_knob("recon_host_reads", ctx=ctx)
    say("async tile", rounds)
    mask, lab, n, hq = rt.rt_segment_tile(rgb, want_hq=True, ctx=ctx)
    emask, elab, en = oracle.segment_from_hq(to_np(hq))
    assert_equal(to_np(lab), elab, f"async labels rounds={rounds}")
    assert_equal(to_np(mask), emask, f"async mask rounds={rounds}")
    assert int(to_np(n)[0]) == en
    assert rt.rt_get_knob("recon_host_reads", ctx=ctx) == reads0
    ctx.close()


def test_async_4k_equals_sync(rt):
    d = dev()
    rgb = to_dev(synth.make_tile(synth.spec_4k(0))[0], d)
    say("sync 4096")
    ref = [to_np(x) for x in rt.rt_segment_tile(rgb)[:3]]
    for rounds in (16, 4):
        ctx = _ctx(rt, recon_async=1, recon_async_rounds=rounds)
        say("async 4096", rounds)
        got = [to_np(x) for x in rt.rt_segment_tile(rgb, ctx=ctx)[:3]]
        assert_equal(got[1], ref[1], f"async 4096 labels rounds={rounds}")
        assert_equal(got[0], ref[0], f"async 4096 mask rounds={rounds}")
        assert int(got[2][0]) == int(ref[2][0])
        ctx.close()


def test_async_batch_and_graph_replays(rt, oracle):
    import torch
    d = dev()
    tiles = [to_dev(synth.make_tile(synth.spec_uneven(i))[0][:900, :700].copy(), d) for i in (2, 5, 9)]
    ref_ctx = rt.Context(0)
    ref = [tuple(to_np(x) for x in o[:3]) for o in rt.rt_segment_batch(tiles, ctx=ref_ctx)]
    ref_ctx.close()
    for graph in (0, 1):
        ctx = _ctx(rt, recon_async=1, recon_async_rounds=6, graph=graph)
        reads0 = rt.rt_get_knob("recon_host_reads", ctx=ctx)
        for rep in range(3):
            say("async batch graph", graph, "rep", rep)
            got = rt.rt_segment_batch(tiles, ctx=ctx)
            torch.cuda.synchronize()
            for i, (g, r) in enumerate(zip(got, ref)):
                assert_equal(to_np(g[1]), r[1], f"graph={graph} rep {rep} tile {i} labels")
                assert_equal(to_np(g[0]), r[0], f"graph={graph} rep {rep} tile {i} mask")
                assert int(to_np(g[2])[0]) == int(r[2][0])
        assert rt.rt_get_knob("recon_host_reads", ctx=ctx) == reads0
        ctx.close()


def test_async_rejects_with_queue_mode(rt):
    d = dev()
    rgb = to_dev(synth.make_tile(synth.spec_small(1))[0], d)
    ctx = _ctx(rt, recon_async=1, recon_mode=1)
    say("async + queue mode falls back to the queue")
    mask, lab, n, hq = rt.rt_segment_tile(rgb, want_hq=True, ctx=ctx)
    ctx2 = rt.Context(0)
    m2, l2, n2 = rt.rt_segment_tile(rgb, ctx=ctx2)[:3]
    assert_equal(to_np(lab), to_np(l2), "queue mode with recon_async set")
    ctx.close()
    ctx2.close()
