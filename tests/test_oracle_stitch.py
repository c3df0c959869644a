"""Pins of the stitching oracle (oracle/stitch_oracle.c) on the CPU: a single
core covering the slide is the plain segmentation of the slide; with no halo
the result is the per-core segmentations re-labelled into slide coordinates
(recomposed here independently, core by core); with a halo wider than a
nucleus, nuclei cut by core borders are recovered, so the stitched slide
agrees with the whole-slide segmentation far better than halo-free tiling
does; every stitched nucleus carries its canonical slide label."""
import numpy as np
import pytest
from scipy import ndimage

from paper_1405_7958_amd import synth


def slide_hq(oracle, w, h, seed):
    spec = synth.TileSpec(w=w, h=h, seed=seed, n_nuclei=int(700 * w * h / 1e6), amin=4, amax=14,
                          cluster_frac=0.2, cluster_min=2, cluster_max=4, jitter=20)
    return oracle.deconv(synth.make_tile(spec)[0])


def test_one_core_is_the_plain_segmentation(oracle):
    hq = slide_hq(oracle, 300, 200, 61000)
    lab, mask, n = oracle.stitch_from_hq(hq, 512, 32)
    elab_mask, elab, en = oracle.segment_from_hq(hq)
    assert np.array_equal(lab, elab) and np.array_equal(mask, elab_mask) and n == en


@pytest.mark.parametrize("tile", [64, 100, 128])
def test_no_halo_is_per_core_segmentation(oracle, tile):
    hq = slide_hq(oracle, 333, 257, 61001)
    H, W = hq.shape
    exp = np.zeros((H, W), np.int32)
    count = 0
    for y0 in range(0, H, tile):
        for x0 in range(0, W, tile):
            sub = np.ascontiguousarray(hq[y0:y0 + tile, x0:x0 + tile])
            _, lab, n = oracle.segment_from_hq(sub)
            count += n
            sh, sw = sub.shape
            ys, xs = np.nonzero(lab)
            root = lab[ys, xs] - 1
            ry, rx = root // sw + y0, root % sw + x0
            exp[ys + y0, xs + x0] = ry * W + rx + 1
    lab, mask, n = oracle.stitch_from_hq(hq, tile, 0)
    assert np.array_equal(lab, exp) and n == count
    assert np.array_equal(mask, (exp > 0).astype(np.uint8))


def _canonical(lab):
    for v in np.unique(lab[lab > 0]):
        ys, xs = np.nonzero(lab == v)
        i = np.argmin(ys * lab.shape[1] + xs)
        assert ys[i] * lab.shape[1] + xs[i] + 1 == v


def _dice(a, b):
    a, b = a > 0, b > 0
    return 2.0 * (a & b).sum() / max(1, a.sum() + b.sum())


@pytest.mark.parametrize("seed", [61002, 61003])
def test_halo_recovers_cut_nuclei(oracle, seed):
    hq = slide_hq(oracle, 520, 390, seed)
    whole_mask, whole, n_whole = oracle.segment_from_hq(hq)
    lab0, _, n0 = oracle.stitch_from_hq(hq, 96, 0)
    lab, mask, n = oracle.stitch_from_hq(hq, 96, 40)
    _canonical(lab)
    # every stitched nucleus is one 8-connected piece
    for v in np.unique(lab[lab > 0])[::5]:
        assert ndimage.label(lab == v, structure=np.ones((3, 3)))[1] == 1
    # the halo recovers the nuclei the core borders cut
    assert _dice(lab, whole) > _dice(lab0, whole)
    assert _dice(lab, whole) >= 0.99 and abs(n - n_whole) <= 2
    assert np.array_equal(mask, (lab > 0).astype(np.uint8))
