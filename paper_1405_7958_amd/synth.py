"""Seeded synthetic H&E-like tissue tiles.

The paper evaluates on 4K x 4K tiles cut from brain-tumour whole-slide images
(Sec. 5, Experimental Results).  Those images are not available, so every input
here is synthetic: a pink background with dark-purple elliptical nuclei, some
isolated and some in touching clusters, plus Gaussian sensor noise.  This module
only draws inputs; it holds none of the segmentation arithmetic, and it is the
one piece of code that both the HIP path's tests and the CPU oracle's tests use.

Recipe (all randomness from ``numpy.random.Generator(PCG64(seed))``):

* background RGB (230, 180, 200); nucleus RGB (120, 70, 150); a low-contrast
  nucleus is halfway between the two, (175, 125, 175);
* per-nucleus integer jitter ``j ~ U{-J..J}`` added to all three channels;
* semi-axes ``a, b ~ U[amin, amax]``, orientation ``theta ~ U[0, pi)``; a pixel
  centre ``(x, y)`` is inside iff
  ``((dx cos t + dy sin t)/a)^2 + ((-dx sin t + dy cos t)/b)^2 <= 1``;
  later nuclei overwrite earlier ones;
* isolated nuclei: centres are rejection-sampled so that circumscribed circles
  keep a gap of at least 2 px to every other nucleus (100 tries, then the
  nucleus is skipped and counted as a shortfall);
* touching clusters: the first member is placed like an isolated nucleus; each
  next member sits in a random direction ``phi`` from a random earlier member at
  distance ``(r1(phi) + r2(phi + pi)) * U[0.6, 0.9]`` (``r(phi)`` = ellipse
  radius along ``phi``), which produces a neck; members keep the 2 px gap to
  nuclei outside their cluster;
* i.i.d. ``N(0, sigma^2)`` noise per pixel and channel after compositing, then
  ``rint``, clip to [0, 255], uint8.

The generator also returns the ground-truth instance map (int32, 0 = background,
k = k-th drawn nucleus), used only for sanity checks (Dice), never for parity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BG_RGB = (230.0, 180.0, 200.0)
NUC_RGB = (120.0, 70.0, 150.0)
LOW_RGB = (175.0, 125.0, 175.0)


@dataclass
class TileSpec:
    w: int
    h: int
    seed: int
    n_nuclei: int
    amin: float = 4.0
    amax: float = 12.0
    cluster_frac: float = 0.15
    cluster_min: int = 2
    cluster_max: int = 2
    jitter: int = 0
    low_contrast: bool = False
    sigma: float = 8.0
    kind: str = "normal"
    extra: dict = field(default_factory=dict)


def _ellipse_radius(a, b, theta, phi):
    c = math.cos(phi - theta)
    s = math.sin(phi - theta)
    return 1.0 / math.sqrt((c / a) ** 2 + (s / b) ** 2)


class _Grid:
    """Uniform hash grid over circle centres for the gap test."""

    def __init__(self, w, h, cell):
        self.cell = max(4.0, float(cell))
        self.nx = int(w // self.cell) + 2
        self.ny = int(h // self.cell) + 2
        self.cells: dict[tuple[int, int], list[int]] = {}
        self.cx: list[float] = []
        self.cy: list[float] = []
        self.r: list[float] = []
        self.group: list[int] = []

    def ok(self, x, y, r, group=-1, gap=2.0):
        cxi = int(x // self.cell)
        cyi = int(y // self.cell)
        reach = int(math.ceil((r + gap + self._rmax) / self.cell)) if self.r else 0
        for gy in range(cyi - reach, cyi + reach + 1):
            for gx in range(cxi - reach, cxi + reach + 1):
                for k in self.cells.get((gx, gy), ()):
                    if group >= 0 and self.group[k] == group:
                        continue
                    d = math.hypot(self.cx[k] - x, self.cy[k] - y)
                    if d < r + self.r[k] + gap:
                        return False
        return True

    _rmax = 0.0

    def add(self, x, y, r, group=-1):
        k = len(self.cx)
        self.cx.append(x)
        self.cy.append(y)
        self.r.append(r)
        self.group.append(group)
        self._rmax = max(self._rmax, r)
        self.cells.setdefault((int(x // self.cell), int(y // self.cell)), []).append(k)


def _draw_layout(spec: TileSpec, rng: np.random.Generator):
    """Returns a list of nuclei (cx, cy, a, b, theta, jitter) and the shortfall."""
    n = spec.n_nuclei
    n_clustered_target = int(round(spec.cluster_frac * n))
    sizes = []
    tot = 0
    while tot < n_clustered_target:
        k = int(rng.integers(spec.cluster_min, spec.cluster_max + 1))
        k = min(k, n_clustered_target - tot)
        if k < 2:
            break
        sizes.append(k)
        tot += k
    n_isolated = n - tot
    grid = _Grid(spec.w, spec.h, 2 * spec.amax + 2)
    nuclei = []
    shortfall = 0

    def shape():
        a = float(rng.uniform(spec.amin, spec.amax))
        b = float(rng.uniform(spec.amin, spec.amax))
        t = float(rng.uniform(0.0, math.pi))
        j = int(rng.integers(-spec.jitter, spec.jitter + 1)) if spec.jitter > 0 else 0
        return a, b, t, j

    def place_free(a, b, group=-1):
        r = max(a, b)
        for _ in range(100):
            x = float(rng.uniform(0, spec.w))
            y = float(rng.uniform(0, spec.h))
            if grid.ok(x, y, r):
                return x, y
        return None

    for gi, k in enumerate(sizes):
        a, b, t, j = shape()
        pos = place_free(a, b)
        if pos is None:
            shortfall += k
            continue
        members = [(pos[0], pos[1], a, b, t, j)]
        grid.add(pos[0], pos[1], max(a, b), group=gi)
        for _m in range(1, k):
            a2, b2, t2, j2 = shape()
            placed = False
            for _ in range(100):
                base = members[int(rng.integers(0, len(members)))]
                phi = float(rng.uniform(0.0, 2.0 * math.pi))
                dist = (_ellipse_radius(base[2], base[3], base[4], phi)
                        + _ellipse_radius(a2, b2, t2, phi + math.pi)) * float(rng.uniform(0.6, 0.9))
                x = base[0] + dist * math.cos(phi)
                y = base[1] + dist * math.sin(phi)
                if not (0 <= x < spec.w and 0 <= y < spec.h):
                    continue
                if grid.ok(x, y, max(a2, b2), group=gi):
                    members.append((x, y, a2, b2, t2, j2))
                    grid.add(x, y, max(a2, b2), group=gi)
                    placed = True
                    break
            if not placed:
                shortfall += 1
        nuclei.extend(members)
    for _ in range(n_isolated):
        a, b, t, j = shape()
        pos = place_free(a, b)
        if pos is None:
            shortfall += 1
            continue
        grid.add(pos[0], pos[1], max(a, b))
        nuclei.append((pos[0], pos[1], a, b, t, j))
    return nuclei, shortfall


def make_tile(spec: TileSpec):
    """Renders one tile.  Returns (rgb uint8 [h, w, 3], gt int32 [h, w], info)."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    nuclei, shortfall = _draw_layout(spec, rng)
    w, h = spec.w, spec.h
    base = LOW_RGB if spec.low_contrast else NUC_RGB
    canvas = np.empty((h, w, 3), np.float32)
    canvas[...] = np.asarray(BG_RGB, np.float32)
    gt = np.zeros((h, w), np.int32)
    for k, (cx, cy, a, b, t, j) in enumerate(nuclei):
        r = max(a, b)
        x0 = max(0, int(math.floor(cx - r)))
        x1 = min(w - 1, int(math.ceil(cx + r)))
        y0 = max(0, int(math.floor(cy - r)))
        y1 = min(h - 1, int(math.ceil(cy + r)))
        if x1 < x0 or y1 < y0:
            continue
        xs = np.arange(x0, x1 + 1, dtype=np.float64) - cx
        ys = np.arange(y0, y1 + 1, dtype=np.float64)[:, None] - cy
        ct, st = math.cos(t), math.sin(t)
        u = (xs * ct + ys * st) / a
        v = (-xs * st + ys * ct) / b
        inside = (u * u + v * v) <= 1.0
        if not inside.any():
            continue
        col = np.asarray(base, np.float32) + np.float32(j)
        sub = canvas[y0:y1 + 1, x0:x1 + 1]
        sub[inside] = col
        gt[y0:y1 + 1, x0:x1 + 1][inside] = k + 1
    noise = rng.standard_normal((h, w, 3), dtype=np.float32) * np.float32(spec.sigma)
    canvas += noise
    np.rint(canvas, out=canvas)
    np.clip(canvas, 0, 255, out=canvas)
    rgb = canvas.astype(np.uint8)
    info = {"n_drawn": len(nuclei), "shortfall": shortfall, "kind": spec.kind}
    return rgb, gt, info


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def spec_small(seed: int = 0) -> TileSpec:
    """512 x 512 tile, ~100 nuclei with semi-axes 4-12 px, ~15% in touching pairs."""
    return TileSpec(w=512, h=512, seed=seed, n_nuclei=100, amin=4, amax=12,
                    cluster_frac=0.15, cluster_min=2, cluster_max=2, jitter=0, kind="small")


def spec_4k(seed: int = 0) -> TileSpec:
    """4096 x 4096 tile, ~8000 nuclei, semi-axes 4-14 px, 20% in clusters of 2-4, jitter +-20."""
    return TileSpec(w=4096, h=4096, seed=seed, n_nuclei=8000, amin=4, amax=14,
                    cluster_frac=0.20, cluster_min=2, cluster_max=4, jitter=20, kind="4k")


_SIZES = (512, 1024, 2048, 4096)


def spec_uneven(i: int, base_seed: int = 1000) -> TileSpec:
    """Tile i of the uneven-size batch: W, H uniform over {512,...,4096}, 300-800 nuclei / Mpx."""
    rng = np.random.Generator(np.random.PCG64(base_seed + i))
    w = int(rng.choice(_SIZES))
    h = int(rng.choice(_SIZES))
    dens = float(rng.uniform(300, 800))
    n = int(round(dens * w * h / 1e6))
    return TileSpec(w=w, h=h, seed=(base_seed + i) * 7919 + 1, n_nuclei=n, amin=4, amax=14,
                    cluster_frac=0.20, cluster_min=2, cluster_max=4, jitter=20, kind="uneven",
                    extra={"density": dens})


def spec_stream(i: int, base_seed: int = 20000) -> TileSpec:
    """Tile i of the mixed stream: 60% normal, 30% dense clustered, 10% low contrast."""
    rng = np.random.Generator(np.random.PCG64(base_seed + i))
    w = int(rng.choice(_SIZES))
    h = int(rng.choice(_SIZES))
    u = float(rng.uniform())
    seed = (base_seed + i) * 7919 + 3
    if u < 0.6:
        dens = float(rng.uniform(300, 800))
        return TileSpec(w=w, h=h, seed=seed, n_nuclei=int(round(dens * w * h / 1e6)), amin=4, amax=14,
                        cluster_frac=0.20, cluster_min=2, cluster_max=4, jitter=20, kind="normal")
    if u < 0.9:
        return TileSpec(w=w, h=h, seed=seed, n_nuclei=int(round(1500 * w * h / 1e6)), amin=4, amax=14,
                        cluster_frac=0.5, cluster_min=3, cluster_max=8, jitter=20, kind="dense")
    dens = float(rng.uniform(300, 800))
    return TileSpec(w=w, h=h, seed=seed, n_nuclei=int(round(dens * w * h / 1e6)), amin=4, amax=14,
                    cluster_frac=0.20, cluster_min=2, cluster_max=4, jitter=10, low_contrast=True,
                    kind="low_contrast")


def random_rgb(h: int, w: int, seed: int) -> np.ndarray:
    """Uniform random RGB bytes (adversarial input for the colour stage)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)


def random_binary(h: int, w: int, p: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((h, w)) < p).astype(np.uint8)


def random_u8(h: int, w: int, seed: int, lo: int = 0, hi: int = 256) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi, size=(h, w), dtype=np.uint8)


def spiral(h: int, w: int, gap: int = 1) -> np.ndarray:
    """Binary spiral corridor of width 1 separated by ``gap`` background pixels:
    one long path, the worst case for wavefront propagation."""
    img = np.zeros((h, w), np.uint8)
    dirs = ((0, 1), (1, 0), (0, -1), (-1, 0))
    y = x = 0
    d = 0
    img[0, 0] = 1

    def can(yy, xx, dy, dx):
        ny, nx = yy + dy, xx + dx
        ay, ax = yy + (gap + 1) * dy, xx + (gap + 1) * dx
        if not (0 <= ny < h and 0 <= nx < w) or img[ny, nx]:
            return False
        if 0 <= ay < h and 0 <= ax < w and img[ay, ax]:
            return False
        return True

    turns = 0
    while True:
        dy, dx = dirs[d]
        if can(y, x, dy, dx):
            y += dy
            x += dx
            img[y, x] = 1
            turns = 0
        else:
            d = (d + 1) % 4
            turns += 1
            if turns > 1:
                break
    return img


def checkerboard(h: int, w: int) -> np.ndarray:
    yy, xx = np.mgrid[0:h, 0:w]
    return ((xx + yy) % 2 == 0).astype(np.uint8)


def nested_rings(h: int, w: int, gap: int = 3) -> np.ndarray:
    yy, xx = np.mgrid[0:h, 0:w]
    cy, cx = (h - 1) / 2.0, (w - 1) / 2.0
    r = np.maximum(np.abs(yy - cy), np.abs(xx - cx)).astype(np.int64)
    return ((r // gap) % 2 == 0).astype(np.uint8)
