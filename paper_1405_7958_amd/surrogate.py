"""Training data, training loop and evaluation of the U-Net surrogate.

The surrogate learns the two maps the plain pipeline hands to its watershed
(Sec. 5.1 segmentation stage): the foreground A after FillHoles and the
first area threshold, and the watershed seeds (regional maxima of the
h-maxima transform of the distance map).  Targets come from the plain
pipeline itself (rt_segment_batch with its foreground / seed outputs) run on
whole synthetic tiles; 512 x 512 training crops are cut from those tiles so
that the crops see the same tile-level context as inference.  The seed
target is the seed map dilated by one 3 x 3 step (thin seeds are hard to hit
exactly; any seed pixel inside a nucleus core identifies the same object).

Every network step runs in the library's kernels (rt_unet_*); this module
only draws inputs, moves tensors and computes evaluation scores.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import rtseg, synth

CROP = 512


def dilate3(m: np.ndarray) -> np.ndarray:
    """3 x 3 binary dilation (in-image neighbours only)."""
    out = m.copy()
    h, w = m.shape
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            ys = slice(max(0, dy), h + min(0, dy))
            yd = slice(max(0, -dy), h + min(0, -dy))
            xs = slice(max(0, dx), w + min(0, dx))
            xd = slice(max(0, -dx), w + min(0, -dx))
            out[yd, xd] |= m[ys, xs]
    return out


def crop_origins(w: int, h: int, rng: np.random.Generator, k: int):
    """k random 512 x 512 crop origins inside a w x h tile (8-aligned)."""
    xs = rng.integers(0, max(1, (w - CROP) // 8 + 1), size=k) * 8
    ys = rng.integers(0, max(1, (h - CROP) // 8 + 1), size=k) * 8
    return list(zip(xs.tolist(), ys.tolist()))


def make_training_set(n_crops: int, base_seed: int = 10000, device=None, ctx=None, workers: int = 8, log=None):
    """n_crops crops of 512 x 512 from tiles of the mixed stream (sizes in
    {512..4096}^2, 60% normal, 30% dense, 10% low contrast), each tile
    segmented by the plain pipeline.  Returns device tensors
    (rgb [n,512,512,3] u8, fg [n,512,512] u8, seeds [n,512,512] u8)."""
    device = device or torch.device("cuda", 0)
    rng = np.random.Generator(np.random.PCG64(base_seed))
    rgb_out = torch.empty((n_crops, CROP, CROP, 3), dtype=torch.uint8, device=device)
    fg_out = torch.empty((n_crops, CROP, CROP), dtype=torch.uint8, device=device)
    sd_out = torch.empty((n_crops, CROP, CROP), dtype=torch.uint8, device=device)
    got = 0
    i = 0
    t0 = time.time()
    with ThreadPoolExecutor(workers) as ex:
        while got < n_crops:
            specs = [synth.spec_stream(base_seed + i + k) for k in range(8)]
            i += 8
            tiles = list(ex.map(lambda s: synth.make_tile(s)[0], specs))
            dev_tiles = [torch.from_numpy(t).to(device) for t in tiles]
            outs = rtseg.rt_segment_batch(dev_tiles, want_maps=True, ctx=ctx)
            for t, dt, o, s in zip(tiles, dev_tiles, outs, specs):
                fg = o[3].cpu().numpy()
                sd = dilate3(o[4].cpu().numpy())
                per = max(1, (s.w * s.h) // (CROP * CROP))
                for ox, oy in crop_origins(s.w, s.h, rng, per):
                    if got >= n_crops:
                        break
                    rgb_out[got] = dt[oy:oy + CROP, ox:ox + CROP]
                    fg_out[got] = torch.from_numpy(np.ascontiguousarray(fg[oy:oy + CROP, ox:ox + CROP])).to(device)
                    sd_out[got] = torch.from_numpy(np.ascontiguousarray(sd[oy:oy + CROP, ox:ox + CROP])).to(device)
                    got += 1
            if log:
                log(f"training crops {got}/{n_crops} ({time.time() - t0:.1f} s)")
    return rgb_out, fg_out, sd_out


def train(net, data, epochs: float = 1.0, batch: int = 8, lr: float = 2e-3, w_seed: float = 1.0, log=None,
          seed: int = 0, time_budget: float | None = None):
    """Adam over shuffled batches; cosine learning-rate decay to lr/20.
    Returns (losses per step, seconds, steps)."""
    rgb, fg, sd = data
    n = rgb.shape[0]
    steps = max(1, int(epochs * n / batch))
    rng = np.random.Generator(np.random.PCG64(seed))
    order = np.concatenate([rng.permutation(n) for _ in range(int(np.ceil(epochs)) + 1)])
    losses = []
    loss = torch.zeros(1, dtype=torch.float32, device=rgb.device)
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(steps):
        idx = torch.from_numpy(order[k * batch:(k + 1) * batch].copy()).to(rgb.device)
        b_rgb = rgb.index_select(0, idx).contiguous()
        b_fg = fg.index_select(0, idx).contiguous()
        b_sd = sd.index_select(0, idx).contiguous()
        cur = lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * k / steps)))
        net.train_step(b_rgb, b_fg, b_sd, lr=cur, w_seed=w_seed, loss=loss)
        losses.append(float(loss.item()))
        if log and (k % 50 == 0 or k == steps - 1):
            log(f"step {k + 1}/{steps} loss {losses[-1]:.4f} lr {cur:.2e} ({time.time() - t0:.1f} s)")
        if time_budget is not None and time.time() - t0 > time_budget:
            break
    torch.cuda.synchronize()
    return losses, time.time() - t0, len(losses)


def dice_iou(a: np.ndarray, b: np.ndarray):
    a = a.astype(bool)
    b = b.astype(bool)
    inter = np.logical_and(a, b).sum()
    sa, sb = a.sum(), b.sum()
    union = sa + sb - inter
    dice = 1.0 if sa + sb == 0 else 2.0 * inter / (sa + sb)
    iou = 1.0 if union == 0 else inter / union
    return float(dice), float(iou)


def evaluate(net, tiles, tau: float, ctx=None, log=None):
    """Surrogate (+ fallback below confidence tau) against the plain pipeline
    on a list of device RGB tiles.  Returns per-tile records and timings."""
    ctx = ctx or net.ctx
    recs = []
    plain = []
    torch.cuda.synchronize()
    t0 = time.time()
    for t in tiles:
        plain.append(rtseg.rt_segment_tile(t, ctx=ctx)[0])
    torch.cuda.synchronize()
    t_plain = time.time() - t0
    sur = []
    t0 = time.time()
    for t in tiles:
        m, l, n, fb, conf = rtseg.rt_segment_tile_surrogate(t, net, tau=tau, ctx=ctx)
        sur.append((m, fb, conf))
    torch.cuda.synchronize()
    t_sur = time.time() - t0
    for k, (p, (m, fb, conf)) in enumerate(zip(plain, sur)):
        d, i = dice_iou(m.cpu().numpy(), p.cpu().numpy())
        recs.append({"tile": k, "h": int(p.shape[0]), "w": int(p.shape[1]), "fallback": fb, "confidence": conf,
                     "dice": d, "iou": i})
    return recs, t_plain, t_sur
