"""U-Net surrogate kernels against the FP64 oracle.

Per layer, both sides get the same bfloat16 activations and weights; the
GPU's float32 results must lie within the worst-case float32 summation bound
of the FP64 result, 2 K 2^-24 sum|a_i b_i| (K = reduction length; products of
bfloat16 values are exact in float32), plus 1e-30.  Max pooling, its
backward pass and the input conversion are compared exactly.
"""
import numpy as np
import pytest

from oracle import unet_oracle as U
from tests.gpu_util import assert_equal, dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu

R = np.random.Generator(np.random.PCG64(11))
U24 = 2.0 ** -24


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()
    return rtseg


def bf16_array(shape, scale=1.0):
    """Random bfloat16 values: (float64 array, uint16 bit patterns)."""
    v = U.bf16_round(R.standard_normal(shape) * scale)
    bits = (v.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return v, bits


def to_dev16(bits, d):
    import torch
    return torch.from_numpy(bits.view(np.int16).copy()).to(d)


def nchw(a):
    return np.ascontiguousarray(a.transpose(0, 3, 1, 2))


def nhwc(a):
    return np.ascontiguousarray(a.transpose(0, 2, 3, 1))


def conv_w_dev_layout(w):
    """oracle [co][ci][3][3] -> device [co][9][ci]"""
    co, ci = w.shape[:2]
    return np.ascontiguousarray(w.reshape(co, ci, 9).transpose(0, 2, 1))


def up_w_dev_layout(w):
    """oracle [ci][co][2][2] -> device [ci][4][co]"""
    ci, co = w.shape[:2]
    return np.ascontiguousarray(w.reshape(ci, co, 4).transpose(0, 2, 1))


def check_close(got, exp, bound, what):
    got = np.asarray(got, np.float64)
    err = np.abs(got - exp)
    bad = err > bound + 1e-30
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} outside the bound; worst err {err.max():.3e}, " \
                          f"bound there {bound.reshape(-1)[np.argmax(err)]:.3e}"


@pytest.mark.parametrize("ci,co,n,h,w", [(8, 16, 1, 7, 9), (16, 32, 2, 12, 20), (64, 128, 1, 6, 10),
                                         (128, 64, 1, 8, 8), (32, 16, 3, 5, 33)])
def test_conv3_forward_and_backward(rt, ci, co, n, h, w):
    import torch
    d = dev()
    x, xb = bf16_array((n, h, w, ci))
    wgt, _ = bf16_array((co, ci, 3, 3), 0.2)
    b = R.standard_normal(co)
    wdev = torch.from_numpy(conv_w_dev_layout(wgt).astype(np.float32)).to(d)
    say("conv3", ci, co, n, h, w)
    wf, wt = rt.nn_pack(0, wdev.reshape(-1), ci, co)
    y = to_np(rt.nn_conv3_fwd(to_dev16(xb, d), wf, torch.from_numpy(b.astype(np.float32)).to(d), co))
    exp = nhwc(U.conv3_fwd(nchw(x), wgt, b.astype(np.float32).astype(np.float64)))
    S = nhwc(U.conv3_fwd(np.abs(nchw(x)), np.abs(wgt), np.abs(b)))
    check_close(y, exp, 2 * (9 * ci + 1) * U24 * S, "conv3 forward")
    # backward with a random bf16 output gradient (the input gradient of the
    # first layer, 8 padded RGB channels, is never needed and not supported)
    g, gb = bf16_array((n, h, w, co))
    dw, db = rt.nn_conv3_wgrad(to_dev16(xb, d), to_dev16(gb, d))
    gx, gw, gbias = U.conv3_bwd(nchw(x), wgt, nchw(g))
    Sx, Sw, _ = U.conv3_bwd(np.abs(nchw(x)), np.abs(wgt), np.abs(nchw(g)))
    if ci % 16 == 0:
        dx = to_np(rt.nn_conv3_dgrad(to_dev16(gb, d), wt, ci))
        check_close(dx, nhwc(gx), 2 * 9 * co * U24 * nhwc(Sx), "conv3 dgrad")
    K = n * h * w
    check_close(to_np(dw), conv_w_dev_layout(gw), 2 * K * U24 * conv_w_dev_layout(Sw), "conv3 wgrad")
    check_close(to_np(db), gbias, 2 * K * U24 * np.abs(g).sum(axis=(0, 1, 2)), "conv3 bias grad")


def test_conv3_relu_concat_and_split(rt):
    import torch
    d = dev()
    n, h, w, c = 2, 10, 14, 16
    x0, x0b = bf16_array((n, h, w, c))
    x1, x1b = bf16_array((n, h, w, c))
    wgt, _ = bf16_array((32, 2 * c, 3, 3), 0.2)
    b = R.standard_normal(32).astype(np.float32).astype(np.float64)
    wdev = torch.from_numpy(conv_w_dev_layout(wgt).astype(np.float32)).to(d)
    wf, wt = rt.nn_pack(0, wdev.reshape(-1), 2 * c, 32)
    say("conv3 concat")
    y = to_np(rt.nn_conv3_fwd(to_dev16(x0b, d), wf, torch.from_numpy(b.astype(np.float32)).to(d), 32, relu=True,
                              x1=to_dev16(x1b, d)))
    xc = np.concatenate([nchw(x0), nchw(x1)], axis=1)
    pre = U.conv3_fwd(xc, wgt, b)
    S = nhwc(U.conv3_fwd(np.abs(xc), np.abs(wgt), np.abs(b)))
    check_close(y, nhwc(U.relu(pre)), 2 * (9 * 2 * c + 1) * U24 * S, "conv3 concat relu")
    g, gb = bf16_array((n, h, w, 32))
    dx0, dx1 = rt.nn_conv3_dgrad(to_dev16(gb, d), wt, 2 * c, c0=c)
    gx, gw, _ = U.conv3_bwd(xc, wgt, nchw(g))
    Sx, Sw, _ = U.conv3_bwd(np.abs(xc), np.abs(wgt), np.abs(nchw(g)))
    check_close(np.concatenate([to_np(dx0), to_np(dx1)], axis=3), nhwc(gx), 2 * 9 * 32 * U24 * nhwc(Sx),
                "conv3 split dgrad")
    dw, _ = rt.nn_conv3_wgrad(to_dev16(x0b, d), to_dev16(gb, d), x1=to_dev16(x1b, d))
    check_close(to_np(dw), conv_w_dev_layout(gw), 2 * n * h * w * U24 * conv_w_dev_layout(Sw), "conv3 concat wgrad")


@pytest.mark.parametrize("ci,co,n,h,w", [(32, 16, 1, 5, 7), (128, 64, 2, 4, 4), (64, 32, 1, 9, 3)])
def test_up2_forward_and_backward(rt, ci, co, n, h, w):
    import torch
    d = dev()
    x, xb = bf16_array((n, h, w, ci))
    wgt, _ = bf16_array((ci, co, 2, 2), 0.2)
    b = R.standard_normal(co).astype(np.float32).astype(np.float64)
    wdev = torch.from_numpy(up_w_dev_layout(wgt).astype(np.float32)).to(d)
    uf, ut = rt.nn_pack(1, wdev.reshape(-1), ci, co)
    say("up2", ci, co, n, h, w)
    y = to_np(rt.nn_up2_fwd(to_dev16(xb, d), uf, torch.from_numpy(b.astype(np.float32)).to(d), co))
    exp = nhwc(U.up2_fwd(nchw(x), wgt, b))
    S = nhwc(U.up2_fwd(np.abs(nchw(x)), np.abs(wgt), np.abs(b)))
    check_close(y, exp, 2 * (ci + 1) * U24 * S, "up2 forward")
    g, gb = bf16_array((n, 2 * h, 2 * w, co))
    dx, dw, db = rt.nn_up2_bwd(to_dev16(xb, d), to_dev16(gb, d), ut)
    gx, gw, gbias = U.up2_bwd(nchw(x), wgt, nchw(g))
    Sx, Sw, _ = U.up2_bwd(np.abs(nchw(x)), np.abs(wgt), np.abs(nchw(g)))
    check_close(to_np(dx), nhwc(gx), 2 * 4 * co * U24 * nhwc(Sx), "up2 dgrad")
    check_close(to_np(dw), up_w_dev_layout(gw), 2 * n * h * w * U24 * up_w_dev_layout(Sw), "up2 wgrad")
    check_close(to_np(db), gbias, 2 * 4 * n * h * w * U24 * np.abs(g).sum(axis=(0, 1, 2)), "up2 bias grad")


def test_pool2_exact_with_ties(rt):
    import torch
    d = dev()
    n, h, w, c = 2, 6, 10, 16
    x = U.bf16_round(np.round(R.standard_normal((n, h, w, c)) * 2) / 2)   # many ties
    xb = (x.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    say("pool2")
    y, idx = rt.nn_pool2_fwd(to_dev16(xb, d))
    ey, eidx = U.pool2_fwd(nchw(x))
    yv = (to_np(y).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert_equal(yv, nhwc(ey), "pool values")
    assert_equal(to_np(idx), nhwc(eidx).astype(np.uint8), "pool argmax")
    dy = R.standard_normal((n, h // 2, w // 2, c)).astype(np.float32)
    base = R.standard_normal((n, h, w, c)).astype(np.float32)
    dx = torch.from_numpy(base.copy()).to(d)
    rt.nn_pool2_bwd(torch.from_numpy(dy).to(d), idx, dx)
    exp = base.astype(np.float64) + nhwc(U.pool2_bwd(nchw(dy.astype(np.float64)), eidx))
    assert_equal(to_np(dx), exp.astype(np.float32), "pool backward")


def test_head_loss(rt):
    import torch
    d = dev()
    n, h, w = 2, 8, 12
    x, xb = bf16_array((n, h, w, 16))
    wh = R.standard_normal((2, 16)).astype(np.float32)
    bh = R.standard_normal(2).astype(np.float32)
    tf = (R.uniform(size=(n, h, w)) > 0.5).astype(np.uint8)
    ts = (R.uniform(size=(n, h, w)) > 0.8).astype(np.uint8)
    say("head loss")
    loss, dx, dw, db = rt.nn_head_loss(to_dev16(xb, d), torch.from_numpy(wh).to(d), torch.from_numpy(bh).to(d),
                                       to_dev(tf, d), to_dev(ts, d), w_seed=0.5)
    z = U.head_fwd(nchw(x), wh.astype(np.float64), bh.astype(np.float64))
    el = U.bce_logits(z[:, 0], tf) + 0.5 * U.bce_logits(z[:, 1], ts)
    gz = np.stack([U.bce_logits_grad(z[:, 0], tf), 0.5 * U.bce_logits_grad(z[:, 1], ts)], axis=1)
    gx, gw, gb = U.head_bwd(nchw(x), wh.astype(np.float64), gz)
    # float32 transcendental evaluation: relative 1e-5 on the mean loss
    assert abs(float(to_np(loss)[0]) - el) <= 1e-5 * max(1.0, abs(el))
    np.testing.assert_allclose(to_np(dx), nhwc(gx), rtol=2e-5, atol=1e-8)
    np.testing.assert_allclose(to_np(dw), gw, rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(to_np(db), gb, rtol=2e-5, atol=1e-7)


def test_prep_input_exhaustive(rt):
    d = dev()
    v = np.arange(256, dtype=np.uint8)
    rgb = np.stack([v, v[::-1], np.roll(v, 7)], axis=1).reshape(16, 16, 3)
    say("prep input")
    x = to_np(rt.nn_prep_input(to_dev(rgb, d)))[0]
    got = (x.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    exp = U.bf16_round(U.prep_input(rgb)[0].transpose(1, 2, 0))
    assert_equal(got[..., :3], exp, "input values")
    assert not got[..., 3:].any()


def _net_params_oracle(vec):
    """device parameter vector -> oracle parameter dict (float64)."""
    P = {}
    off = 0
    for name, sh in U.param_shapes():
        if name.endswith(".w") and len(sh) == 4 and not name.startswith("u"):
            co, ci = sh[0], sh[1]
            cip = 8 if name.startswith("e1a") else ci
            cnt = co * 9 * cip
            dv = vec[off:off + cnt].reshape(co, 9, cip)[:, :, :ci]
            P[name] = dv.transpose(0, 2, 1).reshape(co, ci, 3, 3).astype(np.float64)
        elif name.startswith("u") and name.endswith(".w"):
            ci, co = sh[0], sh[1]
            cnt = ci * 4 * co
            P[name] = vec[off:off + cnt].reshape(ci, 4, co).transpose(0, 2, 1).reshape(ci, co, 2, 2).astype(np.float64)
        else:
            cnt = int(np.prod(sh))
            P[name] = vec[off:off + cnt].reshape(sh).astype(np.float64)
        off += cnt
    assert off == vec.size
    return P


def test_network_forward_and_gradient_vs_oracle(rt):
    """Whole network on a 32 x 32 batch of 2: GPU logits against the oracle
    forward with every activation rounded to bfloat16 like the GPU's; the
    gradient against the FP64 gradient (direction and size)."""
    import torch
    d = dev()
    net = rt.UNet(seed=7)
    vec = net.get_params()
    P = {k: U.bf16_round(v) if k.endswith(".w") else v for k, v in _net_params_oracle(vec).items()}
    rgb = R.integers(0, 256, size=(2, 32, 32, 3), dtype=np.uint8)
    tf = (R.uniform(size=(2, 32, 32)) > 0.6).astype(np.uint8)
    ts = (R.uniform(size=(2, 32, 32)) > 0.9).astype(np.uint8)
    say("unet grad step")
    loss = net.grad_step(to_dev(rgb, d), to_dev(tf, d), to_dev(ts, d), w_seed=1.0)
    G = net.get_grads()
    x = np.concatenate([U.bf16_round(U.prep_input(r)) for r in rgb], axis=0)
    el, EG = U.loss_and_grads(P, x, tf, ts, w_seed=1.0)
    assert abs(float(to_np(loss)[0]) - el) <= 0.02 * abs(el), (float(to_np(loss)[0]), el)
    Gd = _net_params_oracle(G)
    for name in ("e1a.w", "e2b.w", "e4b.w", "u3.w", "d3a.w", "d1b.w", "head.w", "e3a.b", "head.b"):
        a, b = Gd[name].reshape(-1), EG[name].reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))
        assert cos > 0.97, (name, cos)
        assert abs(np.linalg.norm(a) / (np.linalg.norm(b) + 1e-30) - 1) < 0.1, name
    # forward through the tile path (one 32 x 32 window) against the oracle
    # forward with every activation rounded to bfloat16: rounding flips in
    # 17 layers move single logits a little, the maps as a whole stay put
    pf, ps = net.forward(to_dev(rgb[0], d))
    z = U.forward(P, x[:1], round_fn=U.bf16_round)
    sig = 1 / (1 + np.exp(-z[0]))
    for got, exp in ((to_np(pf), sig[0]), (to_np(ps), sig[1])):
        assert np.abs(got - exp).mean() < 2e-3, np.abs(got - exp).mean()
        assert np.abs(got - exp).max() < 2e-2, np.abs(got - exp).max()
    net.close()


def test_training_lowers_the_loss_and_save_load(rt, tmp_path):
    import torch
    d = dev()
    net = rt.UNet(seed=3)
    rgb = R.integers(0, 256, size=(2, 64, 64, 3), dtype=np.uint8)
    tf = (rgb[..., 0] < 100).astype(np.uint8)
    ts = (rgb[..., 1] < 40).astype(np.uint8)
    t = (to_dev(rgb, d), to_dev(tf, d), to_dev(ts, d))
    say("unet train")
    first = float(to_np(net.train_step(*t, lr=3e-3))[0])
    for _ in range(30):
        last = float(to_np(net.train_step(*t, lr=3e-3))[0])
    assert last < 0.7 * first, (first, last)
    p = tmp_path / "net.bin"
    net.save(str(p))
    other = rt.UNet(seed=99)
    other.load(str(p))
    np.testing.assert_array_equal(other.get_params(), net.get_params())
    a = net.forward(t[0][0])
    b = other.forward(t[0][0])
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    net.close()
    other.close()


def test_tile_inference_windows_are_stitched(rt):
    """A 1000 x 700 tile: every output pixel equals the forward pass of the
    512 x 512 window it is taken from, run as a tile of its own."""
    d = dev()
    net = rt.UNet(seed=5)
    img = R.integers(0, 256, size=(700, 1000, 3), dtype=np.uint8)
    say("unet tile windows")
    pf, ps = net.forward(to_dev(img, d))
    pf = to_np(pf)
    # window positions along x: 0, 480 (= 1000 - 512 -> 488); along y: 0, 188
    for ox, oy, xs, ys in [(0, 0, slice(0, 244), slice(0, 350)), (488, 188, slice(745, 1000), slice(350, 700))]:
        w = img[oy:oy + 512, ox:ox + 512].copy()
        wf, _ = net.forward(to_dev(w, d))
        wf = to_np(wf)
        assert_equal(pf[ys, xs], wf[ys.start - oy:ys.stop - oy, xs.start - ox:xs.stop - ox], "window interior")
    net.close()


def test_surrogate_segmentation(rt, oracle):
    """tau > 1 always falls back to the plain pipeline; tau < 0 never does,
    and then the result equals the oracle's fill holes, labelling, area
    threshold, watershed from the network's seeds and final area threshold on
    the thresholded network maps."""
    from paper_1405_7958_amd import synth
    d = dev()
    net = rt.UNet(seed=1)
    rgb, _, _ = synth.make_tile(synth.spec_small(4))
    t = to_dev(rgb, d)
    say("surrogate fallback")
    m, l, n, fb, conf = rt.rt_segment_tile_surrogate(t, net, tau=1.5)
    assert fb
    pm, pl, pn = rt.rt_segment_tile(t)
    assert_equal(to_np(l), to_np(pl), "fallback labels")
    say("surrogate path")
    m, l, n, fb, conf = rt.rt_segment_tile_surrogate(t, net, tau=-1.0)
    assert not fb and 0.0 <= conf <= 1.0
    pf, ps = net.forward(t)
    fg = (to_np(pf) >= 0.5).astype(np.uint8)
    sd = (to_np(ps) >= 0.5).astype(np.uint8)
    F = oracle.fill_holes(fg, 4)
    lab0, _ = oracle.ccl(F, 8)
    _, A, _ = oracle.area_filter(lab0, 20, fg.size)
    wl, _ = oracle.watershed(A, sd)
    elab, emask, k = oracle.area_filter(wl, 20, 1000)
    assert_equal(to_np(l), elab, "surrogate labels")
    assert_equal(to_np(m), emask, "surrogate mask")
    assert int(to_np(n)[0]) == k
    net.close()


def test_plain_pipeline_training_targets(rt, oracle):
    """The foreground A and the seeds the plain pipeline hands to its
    watershed, as returned for training targets, equal the oracle's."""
    from paper_1405_7958_amd import synth
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_stream(3))
    rgb = rgb[:600, :800].copy()
    say("training targets")
    (mask, lab, n, hq, fg, sd), = rt.rt_segment_batch([to_dev(rgb, d)], want_hq=True, want_maps=True)
    _, _, _, inter = oracle.segment_from_hq(to_np(hq), intermediates=True)
    assert_equal(to_np(fg), inter["A"], "foreground A")
    _, _, wi = oracle.watershed(inter["A"], intermediates=True)
    assert_equal(to_np(sd), (wi["seeds"] > 0).astype(np.uint8), "seeds")
