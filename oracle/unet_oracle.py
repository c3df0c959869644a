"""FP64 CPU oracle of the U-Net surrogate (forward, backward, loss, Adam).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

The surrogate stands in for the reconstruction and watershed-seeding steps of
the segmentation stage (Sec. 5.1): a 4-level U-Net (Ronneberger et al. 2015)
with 16/32/64/128 channels maps an RGB tile to two logit maps, foreground and
seeds.  The paper fixes no network, so every definition here is the plain
textbook one, written with numpy in float64, arrays in NCHW order:

  conv3      3x3 cross-correlation with zero padding 1, stride 1, plus bias
  relu       max(x, 0); its derivative is taken as 0 at x == 0
  pool2      2x2 max pooling, stride 2; ties go to the first element of the
             window in row-major order ((0,0), (0,1), (1,0), (1,1))
  up2        2x2 transposed convolution, stride 2 (each input pixel writes a
             2x2 block: y[co, 2i+a, 2j+b] = sum_ci x[ci, i, j] w[ci, co, a, b] + b[co])
  concat     channel concatenation (decoder input first, skip second)
  head       1x1 convolution 16 -> 2 (fg logit, seed logit)
  loss       mean binary cross-entropy with logits of the fg map plus
             w_seed times that of the seed map, means over all pixels
  adam       Kingma & Ba (2015), bias-corrected, no weight decay

Parity of the GPU kernels is per layer: the same bfloat16 inputs and weights
go to both sides, and the GPU's FP32 accumulators are compared with these
FP64 results.
"""
from __future__ import annotations

import numpy as np

CH = (16, 32, 64, 128)
IN_CH = 3


# ----------------------------------------------------------------------------
# layers
# ----------------------------------------------------------------------------

def conv3_fwd(x, w, b):
    """x [N,Ci,H,W], w [Co,Ci,3,3], b [Co] -> [N,Co,H,W]."""
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((n, w.shape[0], h, wd))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], xp[:, :, ky:ky + h, kx:kx + wd])
    return y + b[None, :, None, None]


def conv3_bwd(x, w, gy):
    """Gradients of conv3_fwd: returns (gx, gw, gb)."""
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            gxp[:, :, ky:ky + h, kx:kx + wd] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], gy)
            gw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", gy, xp[:, :, ky:ky + h, kx:kx + wd])
    return gxp[:, :, 1:-1, 1:-1], gw, gy.sum(axis=(0, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def relu_bwd(y, gy):
    """Gradient through relu given its output y (y > 0 <=> input > 0)."""
    return gy * (y > 0)


def pool2_fwd(x):
    """Returns (y, idx) with idx in 0..3 = position of the maximum in the
    window, first in row-major order on ties."""
    n, c, h, w = x.shape
    win = np.stack([x[:, :, a::2, b::2] for a in (0, 1) for b in (0, 1)], axis=0)
    idx = np.argmax(win, axis=0)          # argmax returns the first maximum
    y = np.take_along_axis(win, idx[None], axis=0)[0]
    return y, idx


def pool2_bwd(gy, idx):
    n, c, h, w = gy.shape
    gx = np.zeros((n, c, 2 * h, 2 * w))
    for k, (a, b) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        gx[:, :, a::2, b::2] = gy * (idx == k)
    return gx


def up2_fwd(x, w, b):
    """x [N,Ci,H,W], w [Ci,Co,2,2], b [Co] -> [N,Co,2H,2W]."""
    n, ci, h, wd = x.shape
    y = np.zeros((n, w.shape[1], 2 * h, 2 * wd))
    for a in (0, 1):
        for c in (0, 1):
            y[:, :, a::2, c::2] = np.einsum("co,nchw->nohw", w[:, :, a, c], x)
    return y + b[None, :, None, None]


def up2_bwd(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for a in (0, 1):
        for c in (0, 1):
            g = gy[:, :, a::2, c::2]
            gx += np.einsum("co,nohw->nchw", w[:, :, a, c], g)
            gw[:, :, a, c] = np.einsum("nchw,nohw->co", x, g)
    return gx, gw, gy.sum(axis=(0, 2, 3))


def head_fwd(x, w, b):
    """1x1 convolution: x [N,16,H,W], w [2,16], b [2]."""
    return np.einsum("oc,nchw->nohw", w, x) + b[None, :, None, None]


def head_bwd(x, w, gy):
    return np.einsum("oc,nohw->nchw", w, gy), np.einsum("nohw,nchw->oc", gy, x), gy.sum(axis=(0, 2, 3))


def bce_logits(z, t):
    """Mean binary cross-entropy with logits: max(z,0) - z t + log(1 + e^-|z|)."""
    return float(np.mean(np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))))


def bce_logits_grad(z, t):
    """d mean-BCE / dz = (sigmoid(z) - t) / count."""
    return (1.0 / (1.0 + np.exp(-z)) - t) / z.size


# ----------------------------------------------------------------------------
# the network
# ----------------------------------------------------------------------------

def param_shapes():
    """Ordered list of (name, shape) of every parameter."""
    c1, c2, c3, c4 = CH
    s = []

    def conv(name, ci, co):
        s.append((name + ".w", (co, ci, 3, 3)))
        s.append((name + ".b", (co,)))

    def up(name, ci, co):
        s.append((name + ".w", (ci, co, 2, 2)))
        s.append((name + ".b", (co,)))

    conv("e1a", IN_CH, c1); conv("e1b", c1, c1)
    conv("e2a", c1, c2); conv("e2b", c2, c2)
    conv("e3a", c2, c3); conv("e3b", c3, c3)
    conv("e4a", c3, c4); conv("e4b", c4, c4)
    up("u3", c4, c3); conv("d3a", 2 * c3, c3); conv("d3b", c3, c3)
    up("u2", c3, c2); conv("d2a", 2 * c2, c2); conv("d2b", c2, c2)
    up("u1", c2, c1); conv("d1a", 2 * c1, c1); conv("d1b", c1, c1)
    s.append(("head.w", (2, c1)))
    s.append(("head.b", (2,)))
    return s


def n_params():
    return int(sum(np.prod(sh) for _, sh in param_shapes()))


ENC = (("e1a", "e1b"), ("e2a", "e2b"), ("e3a", "e3b"), ("e4a", "e4b"))
DEC = (("u3", "d3a", "d3b"), ("u2", "d2a", "d2b"), ("u1", "d1a", "d1b"))


def forward(P, x, cache=None, round_fn=None):
    """x [N,3,H,W] (H, W multiples of 8) -> logits [N,2,H,W].

    round_fn, if given, is applied to every stored activation (used to emulate
    a lower-precision activation format)."""
    r = round_fn or (lambda a: a)
    c = {} if cache is None else cache
    h = x
    skips = []
    for lvl, (a, b) in enumerate(ENC):
        c[a + ".in"] = h
        h = r(relu(conv3_fwd(h, P[a + ".w"], P[a + ".b"])))
        c[a + ".out"] = h
        c[b + ".in"] = h
        h = r(relu(conv3_fwd(h, P[b + ".w"], P[b + ".b"])))
        c[b + ".out"] = h
        if lvl < 3:
            skips.append(h)
            h, idx = pool2_fwd(h)
            c["pool%d.idx" % lvl] = idx
    for (u, a, b), skip in zip(DEC, reversed(skips)):
        c[u + ".in"] = h
        h = r(up2_fwd(h, P[u + ".w"], P[u + ".b"]))
        h = np.concatenate([h, skip], axis=1)
        c[a + ".in"] = h
        h = r(relu(conv3_fwd(h, P[a + ".w"], P[a + ".b"])))
        c[a + ".out"] = h
        c[b + ".in"] = h
        h = r(relu(conv3_fwd(h, P[b + ".w"], P[b + ".b"])))
        c[b + ".out"] = h
    c["head.in"] = h
    return head_fwd(h, P["head.w"], P["head.b"])


def loss_and_grads(P, x, t_fg, t_seed, w_seed=1.0):
    """Returns (loss, grads) for targets t_fg, t_seed [N,H,W] in {0,1}."""
    c = {}
    z = forward(P, x, c)
    loss = bce_logits(z[:, 0], t_fg) + w_seed * bce_logits(z[:, 1], t_seed)
    gz = np.stack([bce_logits_grad(z[:, 0], t_fg), w_seed * bce_logits_grad(z[:, 1], t_seed)], axis=1)
    G = {}
    gh, G["head.w"], G["head.b"] = head_bwd(c["head.in"], P["head.w"], gz)
    skip_grads = []              # gradient of the skip halves, level 0 first
    for u, a, b in reversed(DEC):
        gh = relu_bwd(c[b + ".out"], gh)
        gh, G[b + ".w"], G[b + ".b"] = conv3_bwd(c[b + ".in"], P[b + ".w"], gh)
        gh = relu_bwd(c[a + ".out"], gh)
        gh, G[a + ".w"], G[a + ".b"] = conv3_bwd(c[a + ".in"], P[a + ".w"], gh)
        cu = P[u + ".w"].shape[1]
        skip_grads.append(gh[:, cu:])
        gh, G[u + ".w"], G[u + ".b"] = up2_bwd(c[u + ".in"], P[u + ".w"], gh[:, :cu])
    for lvl in (3, 2, 1, 0):
        a, b = ENC[lvl]
        if lvl < 3:
            gh = pool2_bwd(gh, c["pool%d.idx" % lvl]) + skip_grads[lvl]
        gh = relu_bwd(c[b + ".out"], gh)
        gh, G[b + ".w"], G[b + ".b"] = conv3_bwd(c[b + ".in"], P[b + ".w"], gh)
        gh = relu_bwd(c[a + ".out"], gh)
        gh, G[a + ".w"], G[a + ".b"] = conv3_bwd(c[a + ".in"], P[a + ".w"], gh)
    return loss, G


def adam_step(P, G, M, V, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) of every parameter, in place."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] * G[k]
        mh = M[k] / (1 - b1 ** t)
        vh = V[k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)


def init_params(seed):
    """He-normal weights, zero biases (numpy PCG64 stream)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {}
    for name, sh in param_shapes():
        if name.endswith(".b"):
            P[name] = np.zeros(sh)
        else:
            fan_in = sh[1] * sh[2] * sh[3] if len(sh) == 4 and not name.startswith("u") else \
                (sh[0] if name.startswith("u") else sh[1])
            P[name] = rng.standard_normal(sh) * np.sqrt(2.0 / fan_in)
    return P


def bf16_round(a):
    """Round-to-nearest-even of float64 values to bfloat16, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def prep_input(rgb):
    """RGB uint8 [H,W,3] -> network input [1,3,H,W]: value / 255 - 0.5."""
    return (np.asarray(rgb, np.float64).transpose(2, 0, 1)[None] / 255.0) - 0.5
