"""rt_features (per-nucleus shape, intensity, gradient and texture features)
against the CPU oracle, through the C ABI: nucleus labels and every integer
count bit-exact, the FP64 features within 1e-12 relative (both sides
evaluate the same formulas from identical integer counts in the same order;
only the math library's log2, sqrt, exp and atan2 may differ in the last
bit).  Seeded label maps at sizes spanning several 64-pixel row chunks with
ragged tails, the segmentation's own output on the 512 x 512 and
4096 x 4096 workloads, and the edge cases (no nucleus, single pixels in the
tile corners, one nucleus covering the whole tile, fewer output slots than
nuclei, pitched images)."""
import numpy as np
import pytest

from paper_1405_7958_amd import synth
from tests import brute_features as BF
from tests.gpu_util import dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def rt():
    from paper_1405_7958_amd import rtseg
    rtseg.lib()   # fails loudly if the HIP library is missing
    return rtseg


def _compare(rt, oracle, lab, hq, d, what, max_nuclei=65536, pitch=None):
    import torch
    if pitch is None:
        tl, th = to_dev(lab, d), to_dev(hq, d)
    else:
        h, w = lab.shape
        bl = torch.zeros((h, pitch), dtype=torch.int32, device=d)
        bq = torch.zeros((h, pitch + 3), dtype=torch.uint8, device=d)
        bl[:, :w] = to_dev(lab, d)
        bq[:, :w] = to_dev(hq, d)
        tl, th = bl[:, :w], bq[:, :w]
    lo, fo, co, total = rt.rt_features(tl, th, max_nuclei=max_nuclei, want_counts=True)
    elo, efo, eco = oracle.features(lab, hq, want_counts=True)
    assert total == len(elo), (what, total, len(elo))
    k = min(len(elo), max_nuclei)
    assert np.array_equal(to_np(lo), elo[:k]), what
    g_c = to_np(co)
    if not np.array_equal(g_c, eco[:k]):
        bad = np.argwhere(g_c != eco[:k])
        n, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} count mismatches, first nucleus {n} count {c}: "
                             f"{g_c[n, c]} vs {eco[n, c]}")
    g_f = to_np(fo)
    err = np.abs(g_f - efo[:k]) / np.maximum(1.0, np.abs(efo[:k]))
    if err.size and err.max() > TOL:
        n, f = np.unravel_index(np.argmax(err), err.shape)
        raise AssertionError(f"{what}: feature {oracle.FEATURE_NAMES[f]} of nucleus {n}: {g_f[n, f]!r} vs "
                             f"{efo[n, f]!r}")
    return total


@pytest.mark.parametrize("h,w,seed", [(70, 200, 1), (129, 65, 2), (333, 517, 3), (64, 64, 4), (1, 300, 5)])
def test_features_random_label_maps(rt, oracle, h, w, seed):
    d = dev()
    rng = np.random.Generator(np.random.PCG64(900 + seed))
    lab, hq = BF.random_label_map(h, w, rng, n_blobs=max(3, h * w // 400))
    say("features random", h, w, seed)
    _compare(rt, oracle, lab, hq, d, f"random {h}x{w}")


def test_features_segmented_512(rt, oracle):
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    say("features on the segmented 512 tile")
    mask, lab, n, hq = rt.rt_segment_tile(to_dev(rgb, d), want_hq=True)
    total = _compare(rt, oracle, to_np(lab), to_np(hq), d, "segmented 512")
    assert total == int(to_np(n)[0])


def test_features_segmented_4k(rt, oracle):
    d = dev()
    rgb, _, _ = synth.make_tile(synth.spec_4k(0))
    say("features on the segmented 4096 tile")
    mask, lab, n, hq = rt.rt_segment_tile(to_dev(rgb, d), want_hq=True)
    total = _compare(rt, oracle, to_np(lab), to_np(hq), d, "segmented 4096")
    assert total == int(to_np(n)[0]) > 5000


def test_features_edge_cases(rt, oracle):
    d = dev()
    rng = np.random.Generator(np.random.PCG64(950))
    hq = rng.integers(0, 256, size=(90, 130), dtype=np.uint8)
    say("features: no nucleus")
    assert _compare(rt, oracle, np.zeros((90, 130), np.int32), hq, d, "empty") == 0
    say("features: corner pixels")
    lab = np.zeros((90, 130), np.int32)
    for y, x in [(0, 0), (0, 129), (89, 0), (89, 129)]:
        lab[y, x] = y * 130 + x + 1
    assert _compare(rt, oracle, lab, hq, d, "corners") == 4
    say("features: whole tile one nucleus")
    assert _compare(rt, oracle, np.ones((90, 130), np.int32), hq, d, "whole tile") == 1
    say("features: fewer slots than nuclei")
    lab2, hq2 = BF.random_label_map(120, 140, rng, n_blobs=30)
    n = len(np.unique(lab2[lab2 > 0]))
    assert _compare(rt, oracle, lab2, hq2, d, "truncated", max_nuclei=n // 2) == n
    assert _compare(rt, oracle, lab2, hq2, d, "no slots", max_nuclei=0) == n
    say("features: pitched")
    _compare(rt, oracle, lab2, hq2, d, "pitched", pitch=160)
