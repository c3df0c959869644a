"""Pins of the oracle's whole-pipeline composition (segmentation stage of the
paper's example application, Sec. 5.1: ReconToNuclei, FillHoles,
AreaThreshold, BWLabel, Pre-Watershed, Watershed, AreaThreshold).

The composition is re-derived here from pieces that share nothing with the
oracle: reconstruction by threshold decomposition (scipy labelling per level),
scipy's hole filling, canonicalised scipy labelling, np.bincount areas, scipy's
Euclidean distance transform, h-maxima by iterated geodesic dilation, regional
maxima as flat zones without a higher neighbour, the flood re-derived pixel by
pixel from its definition, the cut rule, scipy labelling and inclusive area
bounds.  Element-by-element equality with the oracle on seeded synthetic tiles
and on hand-built images at every threshold edge (component areas 19/20 and
1000/1001, a top-hat equal to the threshold and one below it, a cluster above
the upper bound before the split whose parts are below it) pins the order of
the steps, the comparison operators and the bounds of both area filters.
"""
import math

import numpy as np
import pytest
from scipy import ndimage as ndi

from paper_1405_7958_amd import synth
from tests import brute as B

T_FG, MIN_A, MAX_A, H_SEED = 16, 20, 1000, 3
NEG = -(1 << 40)


def independent_segment(hq, t_fg=T_FG, min_area=MIN_A, max_area=MAX_A, h_seed=H_SEED):
    hq = np.asarray(hq, np.int64)
    h, w = hq.shape
    # ReconToNuclei: reconstruction of the frame marker under Hq, top-hat threshold
    J = np.zeros_like(hq)
    J[0, :], J[-1, :], J[:, 0], J[:, -1] = hq[0, :], hq[-1, :], hq[:, 0], hq[:, -1]
    R = B.recon_threshold_u8(J, hq, conn=8)
    F0 = (hq - R) >= t_fg
    # FillHoles (background 4-connected) and the first area threshold (lower bound only)
    F = ndi.binary_fill_holes(F0)
    L1, _ = B.scipy_ccl(F, 8)
    area1 = np.bincount(L1.ravel(), minlength=h * w + 2)
    A = (L1 > 0) & (area1[L1] >= min_area)
    # distance transform in half-pixel units
    if (~A).any():
        d2 = np.rint(ndi.distance_transform_edt(A) ** 2).astype(np.int64)
        Dq = np.array([math.isqrt(4 * int(v)) for v in d2.ravel()], np.int64).reshape(h, w)
    else:
        Dq = np.full((h, w), 65535, np.int64)
    Dq = np.where(A, Dq, 0)
    if not A.any():
        return np.zeros((h, w), np.uint8), np.zeros((h, w), np.int64), 0
    # seeds: regional maxima of the h-maxima transform on the foreground graph
    g = B.recon_iterate(np.where(A, Dq - h_seed, NEG), np.where(A, Dq, NEG), A)
    rm = B.regional_maxima(g, A) & A
    S, _ = B.scipy_ccl(rm, 8)
    # flooding levels: widest path from the seeds
    lam = B.widest_path(np.where(rm, Dq, NEG), np.where(A, Dq, NEG), A)
    lam = np.where(A, lam, np.iinfo(np.int32).min)
    lab = B.flood_by_definition(A, S, lam)
    # cut: drop a pixel with a smaller nonzero label among its 8 neighbours
    pad = np.pad(lab, 1)
    keep = lab > 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            q = pad[1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
            keep &= ~((q > 0) & (q < lab))
    L2, _ = B.scipy_ccl(keep, 8)
    area2 = np.bincount(L2.ravel(), minlength=h * w + 2)
    ok = (L2 > 0) & (area2[L2] >= min_area) & (area2[L2] <= max_area)
    out = np.where(ok, L2, 0)
    return ok.astype(np.uint8), out, len(np.unique(out[out > 0]))


def _compare(oracle, hq):
    m, lab, n = oracle.segment_from_hq(hq, T_FG, MIN_A, MAX_A, H_SEED)
    em, elab, en = independent_segment(hq)
    assert np.array_equal(lab, elab), "labels differ from the independent composition"
    assert np.array_equal(m, em)
    assert n == en
    return lab, n


def _tiles():
    cases = []
    sizes = [(96, 96), (64, 80), (96, 64), (80, 96), (48, 48)]
    for i in range(22):
        w, h = sizes[i % len(sizes)]
        spec = synth.TileSpec(w=w, h=h, seed=4000 + i, n_nuclei=max(4, w * h // 350), amin=5.0,
                              amax=11.0, cluster_frac=0.7, cluster_min=2, cluster_max=3, jitter=20,
                              low_contrast=(i % 7 == 3))
        cases.append(spec)
    return cases


@pytest.mark.parametrize("spec", _tiles(), ids=lambda s: f"{s.w}x{s.h}-s{s.seed}")
def test_composition_on_seeded_tiles(oracle, spec):
    rgb, _, _ = synth.make_tile(spec)
    hq = oracle.deconv(rgb)
    _compare(oracle, hq)


def _cluster_hq(seed, h=96, w=96):
    """Noisy Hq image with touching clusters of 2-4 discs (necks from centre
    distances (r1 + r2) * U[0.6, 0.8]), so that most components split."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hq = 20 + rng.integers(-3, 4, size=(h, w))
    yy, xx = np.mgrid[0:h, 0:w]
    for _ in range(3):
        cy, cx = rng.integers(22, h - 22), rng.integers(22, w - 22)
        discs = [(cy, cx, rng.uniform(6, 10))]
        for _ in range(int(rng.integers(1, 4))):
            py, px, pr = discs[int(rng.integers(len(discs)))]
            r = rng.uniform(6, 10)
            phi = rng.uniform(0, 2 * np.pi)
            d = (pr + r) * rng.uniform(0.6, 0.8)
            discs.append((py + d * np.sin(phi), px + d * np.cos(phi), r))
        for py, px, r in discs:
            m = (yy - py) ** 2 + (xx - px) ** 2 <= r * r
            hq[m] = 70 + rng.integers(-8, 9, size=int(m.sum()))
    return np.clip(hq, 0, 255).astype(np.uint8)


CLUSTER_SEEDS = range(4100, 4110)


@pytest.mark.parametrize("seed", CLUSTER_SEEDS)
def test_composition_on_touching_clusters(oracle, seed):
    _compare(oracle, _cluster_hq(seed))


def test_cluster_images_exercise_the_split(oracle):
    split = 0
    for seed in CLUSTER_SEEDS:
        _, _, n, I = oracle.segment_from_hq(_cluster_hq(seed), T_FG, MIN_A, MAX_A, H_SEED, intermediates=True)
        _, n_comp = oracle.ccl(I["A"])
        split += n > n_comp    # the watershed split some component of this image
    assert split >= len(CLUSTER_SEEDS) // 2


def _bump_image(h, w, bumps, bg=20):
    """Constant background with flat raised regions: every region's top-hat is
    its height above the background (the reconstruction from the frame stays
    at the background level inside a region that does not reach the frame)."""
    hq = np.full((h, w), bg, np.uint8)
    for mask, height in bumps:
        hq[mask] = bg + height
    return hq


def _rect(h, w, y0, x0, hh, ww):
    m = np.zeros((h, w), bool)
    m[y0:y0 + hh, x0:x0 + ww] = True
    return m


def test_area_bounds_are_inclusive(oracle):
    h, w = 120, 160
    r20 = _rect(h, w, 5, 5, 4, 5)                 # 20 px: kept
    r19 = _rect(h, w, 5, 20, 4, 5)
    r19[5, 20] = False                            # 19 px: below the first threshold
    r1000 = _rect(h, w, 20, 5, 25, 40)            # 1000 px, one flat ridge: one seed, kept
    r1025 = _rect(h, w, 60, 5, 25, 41)            # 1025 px: above the second threshold
    hq = _bump_image(h, w, [(r20, 40), (r19, 40), (r1000, 40), (r1025, 40)])
    lab, n = _compare(oracle, hq)
    assert lab[5, 5] == 5 * w + 5 + 1 and (lab[r20] == lab[5, 5]).all()
    assert (lab[r19] == 0).all()
    assert lab[20, 5] == 20 * w + 5 + 1 and (lab[r1000] == lab[20, 5]).all()
    assert (lab[r1025] == 0).all()
    assert n == 2


def test_tophat_threshold_is_inclusive(oracle):
    h, w = 40, 60
    a = _rect(h, w, 5, 5, 6, 6)
    b = _rect(h, w, 5, 30, 6, 6)
    hq = _bump_image(h, w, [(a, T_FG), (b, T_FG - 1)])
    lab, n = _compare(oracle, hq)
    assert (lab[a] == 5 * w + 5 + 1).all()        # top-hat == t_fg: foreground
    assert (lab[b] == 0).all()                    # one below: background
    assert n == 1


def test_first_area_filter_has_no_upper_bound(oracle):
    # two discs of ~615 px each, joined by a neck: 1 component above 1000 px
    # before the split, two below 1000 after it
    h, w = 64, 96
    yy, xx = np.mgrid[0:h, 0:w]
    d1 = (yy - 32) ** 2 + (xx - 30) ** 2 <= 14 ** 2
    d2 = (yy - 32) ** 2 + (xx - 62) ** 2 <= 14 ** 2
    neck = (np.abs(yy - 32) <= 2) & (xx >= 40) & (xx <= 52)
    comp = d1 | d2 | neck
    assert comp.sum() > 1000
    hq = _bump_image(h, w, [(comp, 50)])
    lab, n = _compare(oracle, hq)
    assert n == 2
    assert lab[32, 30] != lab[32, 62] and lab[32, 30] > 0 and lab[32, 62] > 0


def test_filled_hole_and_frame_contact(oracle):
    h, w = 50, 70
    ring = _rect(h, w, 10, 10, 14, 14) & ~_rect(h, w, 14, 14, 6, 6)   # a ring whose hole is filled
    edge = _rect(h, w, 0, 40, 8, 10)                                   # touches the tile frame
    hq = _bump_image(h, w, [(ring, 40), (edge, 40)])
    lab, _ = _compare(oracle, hq)
    assert (lab[14:20, 14:20] > 0).all()          # the hole belongs to the nucleus
    assert (lab[edge] == 0).all()                 # frame marker reaches it: suppressed


def test_empty_and_all_foreground(oracle):
    _compare(oracle, np.full((24, 30), 20, np.uint8))
    hq = np.full((24, 30), 20, np.uint8)
    hq[1:-1, 1:-1] = 200                           # one large square, everything but the frame
    _compare(oracle, hq)
