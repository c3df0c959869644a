"""Brute-force and library re-derivations used to pin the oracle.

Everything here is written independently of ``oracle/`` from the mathematical
definitions (or from scipy), and is meant for tiny images only.
"""
from __future__ import annotations

from collections import deque

import numpy as np
from scipy import ndimage as ndi

N8 = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
N4 = [(-1, 0), (0, -1), (0, 1), (1, 0)]


def nbrs(conn):
    return N8 if conn == 8 else N4


def recon_iterate(marker, mask, domain=None, conn=8):
    """Reconstruction by iterating R <- max(R, min(dilate(R), mask)) inside the
    domain graph until nothing changes (the geodesic-dilation definition)."""
    mk = np.asarray(marker, np.int64)
    ms = np.asarray(mask, np.int64)
    h, w = ms.shape
    dom = np.ones((h, w), bool) if domain is None else np.asarray(domain).astype(bool)
    R = np.minimum(mk, ms)
    NEG = np.iinfo(np.int64).min // 4
    while True:
        Rn = np.where(dom, R, NEG)
        pad = np.pad(Rn, 1, constant_values=NEG)
        d = Rn.copy()
        for dy, dx in nbrs(conn):
            d = np.maximum(d, pad[1 + dy:1 + dy + h, 1 + dx:1 + dx + w])
        new = np.where(dom, np.maximum(R, np.minimum(d, ms)), R)
        if np.array_equal(new, R):
            return R
        R = new


def recon_threshold_u8(marker, mask, conn=8):
    """u8 reconstruction by threshold decomposition: R(p) = max level l such that
    p is joined, inside {mask >= l}, to a pixel with min(marker,mask) >= l."""
    mk = np.minimum(np.asarray(marker, np.int64), np.asarray(mask, np.int64))
    ms = np.asarray(mask, np.int64)
    st = np.ones((3, 3)) if conn == 8 else None
    R = np.zeros(ms.shape, np.int64)
    for lvl in range(1, 256):
        lab, n = ndi.label(ms >= lvl, structure=st)
        if n == 0:
            break
        hit = np.zeros(n + 1, bool)
        hit[np.unique(lab[(mk >= lvl) & (lab > 0)])] = True
        hit[0] = False
        R[hit[lab]] = lvl
    return R


def canon_labels(lab):
    """Relabels any labelling so that each component carries 1 + its smallest
    row-major index."""
    lab = np.asarray(lab)
    flat = lab.ravel()
    out = np.zeros(flat.shape, np.int64)
    ids = np.unique(flat[flat > 0])
    for i in ids:
        idx = np.flatnonzero(flat == i)
        out[idx] = idx.min() + 1
    return out.reshape(lab.shape)


def scipy_ccl(binary, conn=8):
    st = np.ones((3, 3)) if conn == 8 else None
    lab, n = ndi.label(np.asarray(binary).astype(bool), structure=st)
    return canon_labels(lab), n


def bfs_fill_holes(binary, bg_conn=4):
    b = np.asarray(binary).astype(bool)
    h, w = b.shape
    reach = np.zeros((h, w), bool)
    q = deque()
    for y in range(h):
        for x in range(w):
            if (y in (0, h - 1) or x in (0, w - 1)) and not b[y, x]:
                reach[y, x] = True
                q.append((y, x))
    while q:
        y, x = q.popleft()
        for dy, dx in nbrs(bg_conn):
            yy, xx = y + dy, x + dx
            if 0 <= yy < h and 0 <= xx < w and not b[yy, xx] and not reach[yy, xx]:
                reach[yy, xx] = True
                q.append((yy, xx))
    return (b | ~reach).astype(np.uint8)


def edt_sq_brute(fg):
    fg = np.asarray(fg).astype(bool)
    h, w = fg.shape
    zy, zx = np.nonzero(~fg)
    if len(zy) == 0:
        return np.full((h, w), -1, np.int64)
    yy, xx = np.mgrid[0:h, 0:w]
    d = (yy[..., None] - zy) ** 2 + (xx[..., None] - zx) ** 2
    out = d.min(axis=-1).astype(np.int64)
    out[~fg] = 0
    return out


def widest_path(marker, mask, domain, conn=8):
    """lambda(p) = max over paths of the min along the path, by Bellman-Ford
    style relaxation on the domain graph (same definition as recon)."""
    return recon_iterate(marker, mask, domain, conn)


def regional_maxima(g, domain, conn=8):
    """Flat zones of g inside the domain graph with no strictly higher neighbour."""
    g = np.asarray(g, np.int64)
    dom = np.asarray(domain).astype(bool)
    h, w = g.shape
    seen = np.zeros((h, w), bool)
    rm = np.zeros((h, w), bool)
    for y in range(h):
        for x in range(w):
            if not dom[y, x] or seen[y, x]:
                continue
            zone = [(y, x)]
            seen[y, x] = True
            q = deque([(y, x)])
            higher = False
            while q:
                cy, cx = q.popleft()
                for dy, dx in nbrs(conn):
                    yy, xx = cy + dy, cx + dx
                    if not (0 <= yy < h and 0 <= xx < w) or not dom[yy, xx]:
                        continue
                    if g[yy, xx] > g[cy, cx]:
                        higher = True
                    elif g[yy, xx] == g[cy, cx] and not seen[yy, xx]:
                        seen[yy, xx] = True
                        zone.append((yy, xx))
                        q.append((yy, xx))
            if not higher:
                for cy, cx in zone:
                    rm[cy, cx] = True
    return rm


def flood_by_definition(A, S, lam):
    """Step-8 flood, re-derived per pixel: for every unlabelled p at level L the
    label is the smallest label among the sources (pixels labelled before L) at
    the smallest geodesic distance through U_L.  O(n^2); tiny graphs only."""
    A = np.asarray(A).astype(bool)
    h, w = A.shape
    lab = np.where(A, S, 0).astype(np.int64)
    NEG = np.iinfo(np.int32).min
    levels = sorted({int(v) for v in lam[A & (lab == 0)] if v != NEG}, reverse=True)
    for L in levels:
        U = A & (lab == 0) & (lam == L)
        new = {}
        for (py, px) in zip(*np.nonzero(U)):
            # BFS from p through U; a labelled pixel ends a path
            dist = {(py, px): 0}
            q = deque([(py, px)])
            best_d, best_l = None, None
            while q:
                cy, cx = q.popleft()
                d = dist[(cy, cx)]
                if best_d is not None and d >= best_d:
                    break
                for dy, dx in N8:
                    yy, xx = cy + dy, cx + dx
                    if not (0 <= yy < h and 0 <= xx < w) or not A[yy, xx]:
                        continue
                    if lab[yy, xx] > 0:
                        if best_d is None or d + 1 < best_d:
                            best_d, best_l = d + 1, int(lab[yy, xx])
                        elif d + 1 == best_d:
                            best_l = min(best_l, int(lab[yy, xx]))
                    elif U[yy, xx] and (yy, xx) not in dist:
                        dist[(yy, xx)] = d + 1
                        q.append((yy, xx))
            new[(py, px)] = best_l
        for (py, px), l in new.items():
            assert l is not None, "unreached pixel"
            lab[py, px] = l
    return lab
