"""What training gains: the committed surrogate weights (trained by the
library's own kernels on crops labelled by the plain pipeline) reproduce the
plain pipeline's masks on held-out tiles, an untrained network does not."""
import os

import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests.gpu_util import dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1405_7958_amd",
                       "weights", "unet_surrogate.rtunet")


def dice(a, b):
    a, b = a.astype(bool), b.astype(bool)
    s = a.sum() + b.sum()
    return 1.0 if s == 0 else 2.0 * np.logical_and(a, b).sum() / s


def test_trained_surrogate_matches_plain_on_held_out_tiles():
    from paper_1405_7958_amd import rtseg
    d = dev()
    assert os.path.exists(WEIGHTS), "trained weights missing"
    trained = rtseg.UNet(seed=0)
    trained.load(WEIGHTS)
    untrained = rtseg.UNet(seed=0)
    got_t, got_u = [], []
    for i, (w, h) in enumerate([(1024, 1024), (2048, 512), (700, 900)]):
        spec = synth.TileSpec(w=w, h=h, seed=15000 + 100 + i, n_nuclei=int(600 * w * h / 1e6), amin=4, amax=14,
                              cluster_frac=0.2, cluster_min=2, cluster_max=4, jitter=20)
        t = to_dev(synth.make_tile(spec)[0], d)
        say("surrogate vs plain", w, h)
        plain = to_np(rtseg.rt_segment_tile(t)[0])
        mt, _, _, fb, _ = rtseg.rt_segment_tile_surrogate(t, trained, tau=-1.0)
        mu, _, _, _, _ = rtseg.rt_segment_tile_surrogate(t, untrained, tau=-1.0)
        assert not fb
        got_t.append(dice(to_np(mt), plain))
        got_u.append(dice(to_np(mu), plain))
    assert min(got_t) >= 0.95, got_t
    assert max(got_u) < 0.6, got_u
    trained.close()
    untrained.close()


def test_surrogate_against_the_method_without_it():
    """States what the trained surrogate gains over the plain pipeline alone
    on a held-out 4096 x 4096 tile: agreement (Dice against the plain masks
    and against the generator's ground truth, for both) and speed (tiles/s of
    both, timed on the device after a warm-up).  The assertions bound the
    quality; the speed ratio is printed whatever its sign."""
    import time

    import torch

    from paper_1405_7958_amd import rtseg
    d = dev()
    net = rtseg.UNet(seed=0)
    net.load(WEIGHTS)
    base = synth.spec_4k(0)
    spec = synth.TileSpec(w=4096, h=4096, seed=15100 + 7, n_nuclei=base.n_nuclei, amin=base.amin, amax=base.amax,
                          cluster_frac=base.cluster_frac, cluster_min=base.cluster_min, cluster_max=base.cluster_max,
                          jitter=base.jitter)
    rgb, gt, _ = synth.make_tile(spec)
    t = to_dev(rgb, d)
    say("surrogate vs plain, speed and Dice, 4096x4096")
    plain = rtseg.rt_segment_tile(t)[0]
    sur = rtseg.rt_segment_tile_surrogate(t, net, tau=-1.0)[0]
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        rtseg.rt_segment_tile(t)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        rtseg.rt_segment_tile_surrogate(t, net, tau=-1.0)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / reps
    p, s = to_np(plain), to_np(sur)
    d_sp = dice(s, p)
    d_pg, d_sg = dice(p, gt > 0), dice(s, gt > 0)
    print(f"surrogate vs plain on a held-out 4096x4096 tile: Dice {d_sp:.4f}; against ground truth plain "
          f"{d_pg:.4f}, surrogate {d_sg:.4f}; plain {1 / t_plain:.1f} tiles/s, surrogate {1 / t_sur:.1f} tiles/s, "
          f"speed ratio surrogate/plain {t_plain / t_sur:.3f}", flush=True)
    assert d_sp >= 0.95, d_sp
    assert abs(d_sg - d_pg) <= 0.02, (d_sg, d_pg)
    assert np.isfinite(t_plain) and np.isfinite(t_sur) and t_plain > 0 and t_sur > 0
    net.close()
