"""Independent numpy/scipy re-derivation of the per-nucleus features (test
infrastructure): vectorised over the nucleus' pixel list, with scipy's Sobel
filter and statistics, and the co-occurrence matrix built from shifted
copies of the label map.  Shares nothing with oracle/features_oracle.c."""
import math

import numpy as np
from scipy import ndimage, stats

LEVELS = 16
GBINS = 16
GWIDTH = 32
EDGE_T = 128


def canonical(lab):
    """Relabels every positive label value to 1 + the row-major index of its
    first pixel."""
    out = np.zeros_like(lab, dtype=np.int32)
    flat = lab.ravel()
    vals, first = np.unique(flat, return_index=True)
    for v, f in zip(vals, first):
        if v > 0:
            out.ravel()[flat == v] = f + 1
    return out


def random_label_map(h, w, rng, n_blobs):
    """Foreground = random discs and a few single pixels; each foreground pixel
    takes the nearest of several random seeds (touching nuclei of different
    labels); Hq = background 19 + noise, nuclei 60..140 + noise."""
    yy, xx = np.mgrid[0:h, 0:w]
    fg = np.zeros((h, w), bool)
    for _ in range(n_blobs):
        cy, cx = rng.integers(0, h), rng.integers(0, w)
        r = rng.uniform(1.0, 7.0)
        fg |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    for _ in range(3):
        fg[rng.integers(0, h), rng.integers(0, w)] = True
    seeds = np.argwhere(fg)
    k = min(len(seeds), n_blobs + 3)
    seeds = seeds[rng.choice(len(seeds), size=k, replace=False)]
    d = (yy[..., None] - seeds[:, 0]) ** 2 + (xx[..., None] - seeds[:, 1]) ** 2
    owner = np.argmin(d, axis=2) + 1
    lab = np.where(fg, owner, 0).astype(np.int32)
    base = np.where(fg, 60 + 20 * (owner % 5), 19)
    hq = np.clip(base + rng.integers(-12, 13, size=(h, w)), 0, 255).astype(np.uint8)
    return canonical(lab), hq


def _entropy2(p):
    p = p[p > 0]
    return float(-(p * np.log2(p)).sum())


def nucleus_features(lab, hq, L):
    h, w = lab.shape
    m = lab == L
    ys, xs = np.nonzero(m)
    A = len(ys)
    # perimeter: sides facing another label or the outside
    pad = np.pad(lab, 1, constant_values=0)
    mp = np.pad(m, 1, constant_values=False)
    perim = 0
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        nb = pad[1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
        perim += int((mp[1:-1, 1:-1] & (nb != L)).sum())
    # gradient: scipy's Sobel, replicated borders
    q = hq.astype(np.int64)
    gx = ndimage.sobel(q, axis=1, mode="nearest")
    gy = ndimage.sobel(q, axis=0, mode="nearest")
    g2 = gx * gx + gy * gy
    g = np.array([math.isqrt(int(v)) for v in g2[m]], np.int64)
    ghist = np.bincount(np.minimum(g // GWIDTH, GBINS - 1), minlength=GBINS)
    v = hq[m].astype(np.int64)
    hist = np.bincount(v, minlength=256)
    # co-occurrence from shifted copies: pairs (p, p + (dx, dy)) inside the tile
    ql = (hq // (256 // LEVELS)).astype(np.int64)
    C = np.zeros((LEVELS, LEVELS), np.int64)
    for dx, dy in ((1, 0), (1, 1), (0, 1), (-1, 1)):
        y0, y1 = 0, h - dy
        x0, x1 = max(0, -dx), w - max(0, dx)
        a = m[y0:y1, x0:x1] & (lab[y0 + dy:y1 + dy, x0 + dx:x1 + dx] == L)
        q1 = ql[y0:y1, x0:x1][a]
        q2 = ql[y0 + dy:y1 + dy, x0 + dx:x1 + dx][a]
        np.add.at(C, (q1, q2), 1)
        np.add.at(C, (q2, q1), 1)
    counts = np.concatenate([[A, perim, xs.min(), ys.min(), xs.max(), ys.max()], hist, C.ravel(), ghist,
                             [g.sum(), (g * g).sum(), g.max()]]).astype(np.int64)
    f = {}
    f["area"] = A
    f["perimeter"] = perim
    f["centroid_x"] = xs.mean()
    f["centroid_y"] = ys.mean()
    f["bbox_w"] = xs.max() - xs.min() + 1
    f["bbox_h"] = ys.max() - ys.min() + 1
    f["extent"] = A / (f["bbox_w"] * f["bbox_h"])
    f["equiv_diameter"] = math.sqrt(4 * A / math.pi)
    f["circularity"] = 4 * math.pi * A / perim ** 2
    cov = np.cov(np.vstack([xs, ys]).astype(np.float64), bias=True) + np.eye(2) / 12.0
    ev = np.linalg.eigvalsh(cov)
    l2, l1 = max(ev[0], 0.0), ev[1]
    f["major_axis"] = 4 * math.sqrt(l1)
    f["minor_axis"] = 4 * math.sqrt(l2)
    f["eccentricity"] = math.sqrt(1 - l2 / l1) if l1 > 0 else 0.0
    f["orientation"] = 0.5 * math.atan2(2 * cov[0, 1], cov[0, 0] - cov[1, 1])
    sv = np.sort(v)
    f["int_mean"] = v.mean()
    f["int_std"] = v.std()
    f["int_min"] = v.min()
    f["int_max"] = v.max()
    f["int_median"] = sv[(A - 1) // 2]
    f["int_p25"] = sv[(A - 1) // 4]
    f["int_p75"] = sv[3 * (A - 1) // 4]
    sd = v.std()
    f["int_skewness"] = float(stats.skew(v.astype(np.float64))) if sd > 0 else 0.0
    f["int_kurtosis"] = float(stats.kurtosis(v.astype(np.float64), fisher=False)) if sd > 0 else 0.0
    ph = hist / A
    f["int_entropy"] = _entropy2(ph)
    f["int_energy"] = float((ph ** 2).sum())
    f["int_range"] = v.max() - v.min()
    f["grad_mean"] = g.mean()
    f["grad_std"] = g.std()
    f["grad_max"] = g.max()
    pg = ghist / A
    f["grad_entropy"] = _entropy2(pg)
    f["grad_energy"] = float((pg ** 2).sum())
    f["edge_fraction"] = float((g >= EDGE_T).mean())
    names = ["glcm_asm", "glcm_contrast", "glcm_correlation", "glcm_variance", "glcm_homogeneity",
             "glcm_sum_average", "glcm_sum_variance", "glcm_sum_entropy", "glcm_entropy", "glcm_diff_variance",
             "glcm_diff_entropy", "glcm_imc1", "glcm_imc2", "glcm_max_prob", "glcm_cluster_shade",
             "glcm_cluster_prominence"]
    if C.sum() == 0:
        for n in names:
            f[n] = 0.0
        return counts, f
    p = C / C.sum()
    i, j = np.indices(p.shape)
    px = p.sum(axis=1)
    py = p.sum(axis=0)
    mu = float((np.arange(LEVELS) * px).sum())
    var = float(((np.arange(LEVELS) - mu) ** 2 * px).sum())
    f["glcm_asm"] = float((p ** 2).sum())
    f["glcm_contrast"] = float(((i - j) ** 2 * p).sum())
    f["glcm_correlation"] = float(((i - mu) * (j - mu) * p).sum() / var) if var > 0 else 1.0
    f["glcm_variance"] = var
    f["glcm_homogeneity"] = float((p / (1 + (i - j) ** 2)).sum())
    ps = np.bincount((i + j).ravel(), weights=p.ravel(), minlength=2 * LEVELS - 1)
    pd = np.bincount(np.abs(i - j).ravel(), weights=p.ravel(), minlength=LEVELS)
    k2 = np.arange(2 * LEVELS - 1)
    k1 = np.arange(LEVELS)
    savg = float((k2 * ps).sum())
    f["glcm_sum_average"] = savg
    f["glcm_sum_variance"] = float(((k2 - savg) ** 2 * ps).sum())
    f["glcm_sum_entropy"] = _entropy2(ps)
    hxy = _entropy2(p.ravel())
    f["glcm_entropy"] = hxy
    dm = float((k1 * pd).sum())
    f["glcm_diff_variance"] = float(((k1 - dm) ** 2 * pd).sum())
    f["glcm_diff_entropy"] = _entropy2(pd)
    hx = _entropy2(px)
    pp = np.outer(px, py)
    nz = pp > 0
    hxy1 = float(-(p[nz] * np.log2(pp[nz])).sum())
    hxy2 = float(-(pp[nz] * np.log2(pp[nz])).sum())
    f["glcm_imc1"] = (hxy - hxy1) / hx if hx > 0 else 0.0
    f["glcm_imc2"] = math.sqrt(1 - math.exp(-2 * max(hxy2 - hxy, 0.0)))
    f["glcm_max_prob"] = float(p.max())
    s = i + j - 2 * mu
    f["glcm_cluster_shade"] = float((s ** 3 * p).sum())
    f["glcm_cluster_prominence"] = float((s ** 4 * p).sum())
    return counts, f
