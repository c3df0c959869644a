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
