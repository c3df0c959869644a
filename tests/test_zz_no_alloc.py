"""rt_ccl_noalloc (BWLabel with its scratch in the library's fixed device
array) against rt_ccl, through the C ABI: bit-exact labels and component
counts on two calls in a row, the second on a smaller image, then on a
pitched image and a 4-connected checkerboard (the most components an image
can hold); sizes beyond the array are rejected."""
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


def _both(rt, b, conn, d, pitch=None):
    import torch
    h, w = b.shape
    if pitch is None:
        x = to_dev(b, d)
    else:
        big = torch.zeros((h, pitch), dtype=torch.uint8, device=d)
        big[:, :w] = to_dev(b, d)
        x = big[:, :w]
    ref, nref = rt.rt_ccl(x, conn)
    lab = torch.full((h, x.stride(0)), -7, dtype=torch.int32, device=d)[:, :w]
    n = torch.full((1,), -7, dtype=torch.int32, device=d)
    rt.rt_ccl_noalloc(x, lab, n, conn)
    torch.cuda.synchronize()
    return to_np(lab), int(to_np(n)[0]), to_np(ref), int(to_np(nref)[0])


def test_noalloc_ccl_matches_rt_ccl_twice_then_smaller(rt, oracle):
    d = dev()
    first = synth.random_binary(1500, 1300, 0.45, seed=501)
    second = synth.random_binary(333, 517, 0.55, seed=502)
    for name, b in (("1500x1300", first), ("333x517 after the larger call", second)):
        for conn in (8, 4):
            say("noalloc ccl", name, conn)
            got, n, ref, nref = _both(rt, b, conn, d)
            assert_equal(got, ref, f"noalloc vs rt_ccl {name} conn={conn}")
            assert n == nref
            exp, nexp = oracle.ccl(b, conn)
            assert_equal(got, exp, f"noalloc vs oracle {name} conn={conn}")
            assert n == nexp


def test_noalloc_ccl_pitched_and_checkerboard(rt, oracle):
    d = dev()
    b = synth.random_binary(200, 150, 0.5, seed=503)
    say("noalloc ccl pitched 150x200 pitch 256")
    got, n, ref, nref = _both(rt, b, 8, d, pitch=256)
    assert_equal(got, ref, "noalloc pitched")
    assert n == nref
    chk = synth.checkerboard(100, 99)
    for conn in (4, 8):
        say("noalloc ccl checkerboard", conn)
        got, n, ref, nref = _both(rt, chk, conn, d)
        assert_equal(got, ref, f"noalloc checkerboard conn={conn}")
        exp, nexp = oracle.ccl(chk, conn)
        assert n == nref == nexp


def test_noalloc_ccl_rejects_images_beyond_the_array(rt):
    import torch
    d = dev()
    w, h = 4096, 1025   # one row more than 4 Mpx
    x = torch.zeros((h, w), dtype=torch.uint8, device=d)
    lab = torch.zeros((h, w), dtype=torch.int32, device=d)
    say("noalloc ccl rejects", w, h)
    with pytest.raises(rt.RtError) as ei:
        rt.rt_ccl_noalloc(x, lab)
    assert ei.value.code == rt.RT_EINVAL
    # the library still works after the rejected call
    b = synth.random_binary(64, 64, 0.5, seed=504)
    got, n, ref, nref = _both(rt, b, 8, d)
    assert_equal(got, ref, "noalloc after a rejected call")
