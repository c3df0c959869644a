"""Pins of the feature-computation oracle (oracle/features_oracle.c) on the
CPU: closed forms on shapes whose features follow by hand, invariances, and
an independent numpy/scipy re-derivation of every feature on seeded label
maps (tests/brute_features.py), element by element."""
import math

import numpy as np
import pytest

from tests import brute_features as BF

NAMES = None


@pytest.fixture(scope="module")
def O(oracle):
    global NAMES
    NAMES = oracle.FEATURE_NAMES
    return oracle


def fidx(name):
    return NAMES.index(name)


def feats_of(O, lab, hq):
    lo, fo = O.features(lab, hq)
    return {int(l): dict(zip(O.FEATURE_NAMES, f)) for l, f in zip(lo, fo)}


def test_constant_rectangle_closed_forms(O):
    w, h = 7, 4
    lab = np.zeros((20, 30), np.int32)
    lab[5:5 + h, 10:10 + w] = 5 * 30 + 10 + 1
    hq = np.full((20, 30), 100, np.uint8)   # constant everywhere: zero gradient
    f = feats_of(O, lab, hq)[5 * 30 + 11]
    assert f["area"] == w * h
    assert f["perimeter"] == 2 * (w + h)
    assert f["centroid_x"] == 10 + (w - 1) / 2 and f["centroid_y"] == 5 + (h - 1) / 2
    assert f["bbox_w"] == w and f["bbox_h"] == h and f["extent"] == 1.0
    assert math.isclose(f["circularity"], 4 * math.pi * w * h / (2 * (w + h)) ** 2, rel_tol=1e-14)
    assert math.isclose(f["equiv_diameter"], math.sqrt(4 * w * h / math.pi), rel_tol=1e-14)
    # a w x h block of unit squares: variances w^2/12 and h^2/12, no covariance
    assert math.isclose(f["major_axis"], 4 * math.sqrt(w * w / 12), rel_tol=1e-13)
    assert math.isclose(f["minor_axis"], 4 * math.sqrt(h * h / 12), rel_tol=1e-13)
    assert math.isclose(f["eccentricity"], math.sqrt(1 - (h / w) ** 2), rel_tol=1e-13)
    assert f["orientation"] == 0.0
    for k, v in [("int_mean", 100), ("int_std", 0), ("int_min", 100), ("int_max", 100), ("int_median", 100),
                 ("int_p25", 100), ("int_p75", 100), ("int_skewness", 0), ("int_kurtosis", 0),
                 ("int_entropy", 0), ("int_energy", 1), ("int_range", 0), ("grad_mean", 0), ("grad_std", 0),
                 ("grad_max", 0), ("grad_entropy", 0), ("grad_energy", 1), ("edge_fraction", 0),
                 ("glcm_asm", 1), ("glcm_contrast", 0), ("glcm_correlation", 1), ("glcm_variance", 0),
                 ("glcm_homogeneity", 1), ("glcm_sum_average", 2 * (100 // 16)), ("glcm_sum_variance", 0),
                 ("glcm_sum_entropy", 0), ("glcm_entropy", 0), ("glcm_diff_variance", 0),
                 ("glcm_diff_entropy", 0), ("glcm_imc1", 0), ("glcm_imc2", 0), ("glcm_max_prob", 1),
                 ("glcm_cluster_shade", 0), ("glcm_cluster_prominence", 0)]:
        assert f[k] == v, (k, f[k], v)


def test_striped_rectangle_cooccurrence_closed_form(O):
    """Columns alternate between two grey levels two quantisation levels
    apart: horizontal and diagonal pairs differ, vertical pairs agree."""
    w, h = 9, 6
    lab = np.zeros((16, 16), np.int32)
    lab[3:3 + h, 4:4 + w] = 3 * 16 + 4 + 1
    hq = np.zeros((16, 16), np.uint8)
    hq[:, 0::2] = 16    # level 1
    hq[:, 1::2] = 48    # level 3
    _, _, counts = O.features(lab, hq, want_counts=True)
    C = counts[0, 262:262 + 256].reshape(16, 16)
    n_h, n_v, n_d = (w - 1) * h, w * (h - 1), 2 * (w - 1) * (h - 1)
    assert C.sum() == 2 * (n_h + n_v + n_d)
    assert C[1, 3] == C[3, 1] == n_h + n_d
    assert C[1, 1] + C[3, 3] == 2 * n_v
    f = feats_of(O, lab, hq)[3 * 16 + 5]
    tot = 2 * (n_h + n_v + n_d)
    assert math.isclose(f["glcm_contrast"], 4 * 2 * (n_h + n_d) / tot, rel_tol=1e-14)
    assert math.isclose(f["glcm_homogeneity"], (2 * n_v + 2 * (n_h + n_d) / 5) / tot, rel_tol=1e-14)
    assert math.isclose(f["glcm_diff_variance"],
                        (lambda pd: pd * (1 - pd) * 4)(2 * (n_h + n_d) / tot), rel_tol=1e-13)


def test_single_pixel_nucleus(O):
    lab = np.zeros((5, 5), np.int32)
    lab[2, 3] = 2 * 5 + 3 + 1
    hq = np.full((5, 5), 40, np.uint8)
    f = feats_of(O, lab, hq)[14]
    assert f["area"] == 1 and f["perimeter"] == 4
    assert math.isclose(f["circularity"], math.pi / 4, rel_tol=1e-15)
    assert math.isclose(f["major_axis"], 4 * math.sqrt(1 / 12), rel_tol=1e-14)
    assert f["major_axis"] == f["minor_axis"] and f["eccentricity"] == 0.0
    assert all(f[k] == 0 for k in NAMES if k.startswith("glcm_"))


def test_perimeter_counts_tile_edge_and_neighbour_sides(O):
    lab = np.zeros((5, 6), np.int32)
    lab[0:3, 0:3] = 1            # 3 x 3 in the corner: all 12 outer sides count
    lab[0:2, 3:5] = 4            # touches the first one along two sides
    hq = np.full((5, 6), 50, np.uint8)
    f = feats_of(O, lab, hq)
    assert f[1]["perimeter"] == 12
    assert f[4]["perimeter"] == 8


def test_diagonal_line_orientation(O):
    n = 10
    lab = np.zeros((12, 12), np.int32)
    for i in range(n):
        lab[1 + i, 1 + i] = 1 * 12 + 1 + 1
    hq = np.full((12, 12), 90, np.uint8)
    f = feats_of(O, lab, hq)[14]
    assert math.isclose(f["orientation"], math.pi / 4, rel_tol=1e-14)   # down-right, y down
    assert f["perimeter"] == 4 * n
    # variances (n^2 - 1)/12 + 1/12 on both axes, covariance (n^2 - 1)/12
    var, cov = n * n / 12, (n * n - 1) / 12
    assert math.isclose(f["major_axis"], 4 * math.sqrt(var + cov), rel_tol=1e-13)
    assert math.isclose(f["minor_axis"], 4 * math.sqrt(var - cov), rel_tol=1e-13)


def test_sobel_step_edge(O):
    hq = np.zeros((8, 8), np.uint8)
    hq[:, 4:] = 100
    assert O.sobel_mag(hq, 4, 4) == 400 and O.sobel_mag(hq, 3, 4) == 400
    assert O.sobel_mag(hq, 1, 4) == 0 and O.sobel_mag(hq, 6, 0) == 0
    # replicated borders: the corner sees its own row and column repeated
    hq2 = np.arange(64, dtype=np.uint8).reshape(8, 8)
    gx = (hq2[0, 1] - hq2[0, 0]) * 3 + (hq2[1, 1] - hq2[1, 0])
    gy = (hq2[1, 0] - hq2[0, 0]) * 3 + (hq2[1, 1] - hq2[0, 1])
    assert O.sobel_mag(hq2, 0, 0) == math.isqrt(int(gx) ** 2 + int(gy) ** 2)


def test_translation_and_transposition(O):
    rng = np.random.Generator(np.random.PCG64(7))
    lab, hq = BF.random_label_map(40, 36, rng, n_blobs=6)
    base = dict(zip(*O.features(lab, hq)))
    # transposition: shape features swap axes; intensity, gradient and pooled
    # texture features are unchanged (the offset set maps onto itself)
    labT = BF.canonical(np.ascontiguousarray(lab.T))
    hqT = np.ascontiguousarray(hq.T)
    lo, fo = O.features(labT, hqT)
    i = {k: fidx(k) for k in NAMES}
    # match nuclei by their pixel sets
    for l2, f2 in zip(lo, fo):
        ys, xs = np.nonzero(labT == l2)
        l1 = int(lab[xs[0], ys[0]])
        f1 = base[l1]
        for k in NAMES:
            if k in ("centroid_x", "centroid_y", "bbox_w", "bbox_h", "orientation"):
                continue
            assert math.isclose(f1[i[k]], f2[i[k]], rel_tol=1e-12, abs_tol=1e-12), k
        assert f1[i["centroid_x"]] == f2[i["centroid_y"]] and f1[i["bbox_w"]] == f2[i["bbox_h"]]
    # translation away from the tile edge: everything but the centroid is equal
    big = np.zeros((60, 70), np.int32)
    bighq = np.full((60, 70), 19, np.uint8)
    big[10:10 + lab.shape[0], 20:20 + lab.shape[1]] = lab
    bighq[10:10 + lab.shape[0], 20:20 + lab.shape[1]] = hq
    big = BF.canonical(big)
    # the original map's outer frame holds background at Hq 19 around it
    small = np.zeros((lab.shape[0] + 2, lab.shape[1] + 2), np.int32)
    smallhq = np.full(small.shape, 19, np.uint8)
    small[1:-1, 1:-1] = lab
    smallhq[1:-1, 1:-1] = hq
    small = BF.canonical(small)
    fa = dict(zip(*O.features(small, smallhq)))
    fb = dict(zip(*O.features(big, bighq)))
    for la, f1 in fa.items():
        ys, xs = np.nonzero(small == la)
        f2 = fb[int(big[ys[0] + 9, xs[0] + 19])]
        for k in NAMES:
            if k in ("centroid_x", "centroid_y"):
                continue
            assert f1[i[k]] == f2[i[k]], k
        assert f2[i["centroid_x"]] - f1[i["centroid_x"]] == pytest.approx(19, abs=1e-9)


@pytest.mark.parametrize("seed", range(8))
def test_features_against_independent_rederivation(O, seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    h, w = int(rng.integers(20, 70)), int(rng.integers(20, 70))
    lab, hq = BF.random_label_map(h, w, rng, n_blobs=int(rng.integers(3, 12)))
    lo, fo, co = O.features(lab, hq, want_counts=True)
    exp_labels = np.unique(lab[lab > 0])
    assert np.array_equal(lo, exp_labels)
    for l, f, c in zip(lo, fo, co):
        ref_counts, ref = BF.nucleus_features(lab, hq, int(l))
        assert np.array_equal(c, ref_counts), l
        for k, name in enumerate(NAMES):
            assert math.isclose(f[k], ref[name], rel_tol=1e-10, abs_tol=1e-10), (seed, l, name, f[k], ref[name])


def test_features_on_the_segmented_512_tile(O):
    """The segmentation's own labels (canonical, connected) and Hq."""
    from paper_1405_7958_amd import synth
    rgb, _, _ = synth.make_tile(synth.spec_small(0))
    hq = O.deconv(rgb)
    _, lab, n = O.segment_from_hq(hq)
    lo, fo, co = O.features(lab, hq, want_counts=True)
    assert len(lo) == n
    for l, f, c in list(zip(lo, fo, co))[::9]:
        ref_counts, ref = BF.nucleus_features(lab, hq, int(l))
        assert np.array_equal(c, ref_counts)
        for k, name in enumerate(NAMES):
            assert math.isclose(f[k], ref[name], rel_tol=1e-10, abs_tol=1e-10), (l, name)
