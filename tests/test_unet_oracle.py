"""Pins of the FP64 U-Net oracle: brute force, closed forms, library special
cases and central finite differences (no GPU)."""
import numpy as np
import pytest

from oracle import unet_oracle as U

R = np.random.Generator(np.random.PCG64(5))


def brute_conv3(x, w, b):
    n, ci, h, wd = x.shape
    co = w.shape[0]
    y = np.zeros((n, co, h, wd))
    for a in range(n):
        for o in range(co):
            for i in range(h):
                for j in range(wd):
                    s = b[o]
                    for c in range(ci):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xx = i + ky - 1, j + kx - 1
                                if 0 <= yy < h and 0 <= xx < wd:
                                    s += w[o, c, ky, kx] * x[a, c, yy, xx]
                    y[a, o, i, j] = s
    return y


def fd_check(f, x, g, n=12, eps=1e-6, tol=1e-6):
    """Central differences of scalar f at n random entries of x against g."""
    flat = x.reshape(-1)
    for k in R.choice(flat.size, size=min(n, flat.size), replace=False):
        old = flat[k]
        flat[k] = old + eps
        fp = f()
        flat[k] = old - eps
        fm = f()
        flat[k] = old
        num = (fp - fm) / (2 * eps)
        assert abs(num - g.reshape(-1)[k]) <= tol * max(abs(num), 1.0), (k, num, g.reshape(-1)[k])


def test_conv3_matches_brute_force():
    x = R.standard_normal((2, 3, 5, 7))
    w = R.standard_normal((4, 3, 3, 3))
    b = R.standard_normal(4)
    np.testing.assert_allclose(U.conv3_fwd(x, w, b), brute_conv3(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv3_single_channel_is_correlate2d():
    from scipy.signal import correlate2d
    x = R.standard_normal((1, 1, 9, 6))
    w = R.standard_normal((1, 1, 3, 3))
    ref = correlate2d(x[0, 0], w[0, 0], mode="same", boundary="fill", fillvalue=0.0)
    np.testing.assert_allclose(U.conv3_fwd(x, w, np.zeros(1))[0, 0], ref, rtol=1e-12, atol=1e-12)


def test_conv3_delta_kernels_shift():
    x = R.standard_normal((1, 2, 6, 6))
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 1, 1] = 1.0          # identity on channel 0
    w[1, 1, 0, 2] = 1.0          # y[i, j] = x[i-1, j+1]
    y = U.conv3_fwd(x, w, np.array([0.0, 0.5]))
    np.testing.assert_array_equal(y[0, 0], x[0, 0])
    exp = np.full((6, 6), 0.5)
    exp[1:, :-1] += x[0, 1, :-1, 1:]
    np.testing.assert_allclose(y[0, 1], exp, rtol=0, atol=1e-15)


def test_conv3_bwd_finite_differences():
    x = R.standard_normal((2, 3, 5, 4))
    w = R.standard_normal((4, 3, 3, 3))
    b = R.standard_normal(4)
    gy = R.standard_normal((2, 4, 5, 4))
    f = lambda: float(np.sum(U.conv3_fwd(x, w, b) * gy))
    gx, gw, gb = U.conv3_bwd(x, w, gy)
    fd_check(f, x, gx)
    fd_check(f, w, gw)
    fd_check(f, b, gb)


def test_pool2_ties_and_values():
    x = np.array([[[[1., 1., 0., 5.],
                    [1., 1., 5., 5.],
                    [2., 3., 7., 7.],
                    [4., 4., 7., 9.]]]])
    y, idx = U.pool2_fwd(x)
    np.testing.assert_array_equal(y[0, 0], [[1, 5], [4, 9]])
    np.testing.assert_array_equal(idx[0, 0], [[0, 1], [2, 3]])
    gy = np.array([[[[10., 20.], [30., 40.]]]])
    gx = U.pool2_bwd(gy, idx)
    assert gx.sum() == gy.sum()
    assert gx[0, 0, 0, 0] == 10 and gx[0, 0, 0, 3] == 20 and gx[0, 0, 3, 0] == 30 and gx[0, 0, 3, 3] == 40


def test_pool2_bwd_finite_differences():
    x = R.standard_normal((1, 3, 6, 8))        # continuous values: no ties
    gy = R.standard_normal((1, 3, 3, 4))
    f = lambda: float(np.sum(U.pool2_fwd(x)[0] * gy))
    fd_check(f, x, U.pool2_bwd(gy, U.pool2_fwd(x)[1]))


def test_up2_single_channel_is_kron():
    x = R.standard_normal((1, 1, 3, 4))
    w = R.standard_normal((1, 1, 2, 2))
    y = U.up2_fwd(x, w, np.array([0.25]))
    np.testing.assert_allclose(y[0, 0], np.kron(x[0, 0], w[0, 0]) + 0.25, rtol=1e-13, atol=1e-13)


def test_up2_and_head_bwd_finite_differences():
    x = R.standard_normal((2, 3, 3, 2))
    w = R.standard_normal((3, 4, 2, 2))
    b = R.standard_normal(4)
    gy = R.standard_normal((2, 4, 6, 4))
    f = lambda: float(np.sum(U.up2_fwd(x, w, b) * gy))
    gx, gw, gb = U.up2_bwd(x, w, gy)
    fd_check(f, x, gx)
    fd_check(f, w, gw)
    fd_check(f, b, gb)
    xh = R.standard_normal((1, 16, 3, 3))
    wh = R.standard_normal((2, 16))
    bh = R.standard_normal(2)
    gh = R.standard_normal((1, 2, 3, 3))
    fh = lambda: float(np.sum(U.head_fwd(xh, wh, bh) * gh))
    gxh, gwh, gbh = U.head_bwd(xh, wh, gh)
    fd_check(fh, xh, gxh)
    fd_check(fh, wh, gwh)
    fd_check(fh, bh, gbh)


def test_bce_closed_forms_and_gradient():
    z = np.zeros((3, 4))
    t = (R.uniform(size=(3, 4)) > 0.5).astype(float)
    assert abs(U.bce_logits(z, t) - np.log(2.0)) < 1e-15
    assert abs(U.bce_logits(np.array([40.0]), np.array([1.0]))) < 1e-15
    assert abs(U.bce_logits(np.array([-40.0]), np.array([1.0])) - 40.0) < 1e-12
    z = R.standard_normal((2, 5)) * 3
    t2 = (R.uniform(size=(2, 5)) > 0.5).astype(float)
    f = lambda: U.bce_logits(z, t2)
    fd_check(f, z, U.bce_logits_grad(z, t2))


def test_bf16_round_matches_torch_and_ties_to_even():
    import torch
    v = np.concatenate([R.standard_normal(5000) * 10 ** R.uniform(-6, 6, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -0.0, 65504.0, 3.0e38]])
    exp = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.bf16_round(v), exp)
    assert U.bf16_round(1 + 2 ** -8) == 1.0
    assert U.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_param_count():
    # 3x3 weights: 3*16*9 + 16*16*9 + 16*32*9 + 32*32*9 + 32*64*9 + 64*64*9 + 64*128*9 + 128*128*9
    #   + 128*64*9 + 64*64*9 + 64*32*9 + 32*32*9 + 32*16*9 + 16*16*9 = 438192
    # 2x2 up-convolutions: 128*64*4 + 64*32*4 + 32*16*4 = 43008; head 16*2 = 32; biases 818
    assert U.n_params() == 438192 + 43008 + 32 + 818 == 482050


def test_unet_gradients_finite_differences():
    P = U.init_params(3)
    x = R.standard_normal((1, 3, 8, 8)) * 0.5
    t_fg = (R.uniform(size=(1, 8, 8)) > 0.5).astype(float)
    t_seed = (R.uniform(size=(1, 8, 8)) > 0.8).astype(float)
    loss, G = U.loss_and_grads(P, x, t_fg, t_seed, w_seed=0.7)

    def f():
        z = U.forward(P, x)
        return U.bce_logits(z[:, 0], t_fg) + 0.7 * U.bce_logits(z[:, 1], t_seed)

    assert abs(f() - loss) < 1e-12
    for name in ("e1a.w", "e2b.b", "e4b.w", "u3.w", "d3a.w", "u1.b", "d1b.w", "head.w", "head.b"):
        fd_check(f, P[name], G[name], n=4, eps=1e-5, tol=1e-5)


def test_adam_first_step_closed_form():
    P = {"a": np.array([1.0, -2.0, 3.0])}
    G = {"a": np.array([0.5, -4.0, 1e-3])}
    M = {"a": np.zeros(3)}
    V = {"a": np.zeros(3)}
    U.adam_step(P, G, M, V, 1, lr=0.01)
    # first bias-corrected step: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    exp = np.array([1.0, -2.0, 3.0]) - 0.01 * G["a"] / (np.abs(G["a"]) + 1e-8)
    np.testing.assert_allclose(P["a"], exp, rtol=1e-14)


def test_adam_constant_gradient_every_step():
    # with g constant, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected step is lr * g / (|g| + eps) at every t: pins both
    # corrections (a missing or wrong power of beta shows from t = 2 on)
    g = np.array([0.5, -4.0, 1e-3, 7.0])
    P = {"a": np.zeros(4)}
    M = {"a": np.zeros(4)}
    V = {"a": np.zeros(4)}
    step = 0.01 * g / (np.abs(g) + 1e-8)
    for t in range(1, 51):
        before = P["a"].copy()
        U.adam_step(P, {"a": g}, M, V, t, lr=0.01)
        np.testing.assert_allclose(before - P["a"], step, rtol=1e-9, atol=1e-15)


def test_adam_two_steps_by_hand():
    # g1 = 1, g2 = -3, p0 = 0.5, lr = 0.1, betas (0.9, 0.999), eps 1e-8, worked
    # out by hand in 40-digit decimal arithmetic:
    #   t=1: m = 0.1, v = 0.001, m^ = 1, v^ = 1, p = 0.5 - 0.1 / (1 + 1e-8)
    #   t=2: m = 0.09 - 0.3 = -0.21, v = 0.000999 + 0.009 = 0.009999,
    #        m^ = -0.21 / 0.19, v^ = 0.009999 / 0.001999,
    #        p = p1 - 0.1 * m^ / (sqrt(v^) + 1e-8)
    P = {"a": np.array([0.5])}
    M = {"a": np.zeros(1)}
    V = {"a": np.zeros(1)}
    U.adam_step(P, {"a": np.array([1.0])}, M, V, 1, lr=0.1)
    assert abs(P["a"][0] - 0.40000000099999999) < 1e-15
    U.adam_step(P, {"a": np.array([-3.0])}, M, V, 2, lr=0.1)
    assert abs(M["a"][0] - (-0.21)) < 1e-15 and abs(V["a"][0] - 0.009999) < 1e-16
    assert abs(P["a"][0] - 0.44941898410874449) < 1e-14


def test_adam_scale_and_sign_symmetry():
    # with eps negligible the update depends on the gradient history only
    # through m / sqrt(v): scaling every gradient by c > 0 leaves it unchanged,
    # flipping every sign flips it
    r = np.random.Generator(np.random.PCG64(11))
    gs = [r.standard_normal(6) for _ in range(5)]

    def run(scale):
        P = {"a": np.zeros(6)}
        M = {"a": np.zeros(6)}
        V = {"a": np.zeros(6)}
        for t, g in enumerate(gs, 1):
            U.adam_step(P, {"a": g * scale}, M, V, t, lr=0.01, eps=0.0)
        return P["a"]

    np.testing.assert_allclose(run(1.0), run(37.0), rtol=1e-12)
    np.testing.assert_allclose(run(1.0), -run(-1.0), rtol=1e-12)
