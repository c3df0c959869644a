"""Autotuner for the segmentation launch knobs of a context.

The knobs (rt_set_knob) change only speed, never results: the number of
threshold levels of the connectivity bound that seeds ReconToNuclei, the
propagation rounds launched between two host checks, the in-tile sweep
budget, the routing of components to the per-object kernels, and whether a
batch replays from captured HIP graphs (with how many reconstruction rounds
inside the first graph).  The tuner times
rt_segment_batch on a sample of the caller's own tiles with coordinate
descent over those knobs and keeps the fastest setting, cached in a JSON file
keyed by device and tile-size signature.

The tile shapes of the kernels themselves are fixed by the 64-lane wave
(64 x 64 CCL tiles, 62 x 62 reconstruction interiors with a one-pixel halo
ring, 32 x 32 and 64 x 64 per-object crops in LDS), so they are not searched.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import rtseg

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

SPACE = {
    "recon_level_mode": [1, 0],
    "recon_level_frac": [500, 450, 550, 400, 600],
    "recon_levels": [2, 1, 3, 4, 6, 8, 0],
    "recon_round_batch": [4, 5, 6, 8, 16, 32],
    "recon_max_sweeps": [16, 32, 64, 128],
    "objects_path": [0],
    "recon_mode": [0, 1, 2],
    "recon_queue_after": [2, 1, 3, 4],
}


def signature(rgbs) -> str:
    """Device name and the multiset of tile sizes (sorted)."""
    sizes = sorted((int(t.shape[1]), int(t.shape[0])) for t in rgbs)
    name = torch.cuda.get_device_name(rgbs[0].device) if rgbs else "none"
    return f"{name}|" + ",".join(f"{w}x{h}" for w, h in sizes)


def _time(fn, reps: int) -> float:
    """Median milliseconds of fn() over `reps` runs (after one warm-up)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def apply(knobs: dict, ctx=None):
    for k, v in knobs.items():
        rtseg.rt_set_knob(k, int(v), ctx=ctx)


def current(ctx=None) -> dict:
    return {k: rtseg.rt_get_knob(k, ctx=ctx) for k in rtseg.KNOBS}


def autotune(rgbs, params=None, ctx=None, reps: int = 5, cache: str | None = DEFAULT_CACHE, verbose=False,
             allow_graph: bool = True, trials: bool = True) -> dict:
    """Tunes the knobs of `ctx` for batches like `rgbs` (a list of device
    tiles) and leaves the best setting applied.  Returns
    {"knobs": ..., "ms": ..., "trials": [...]}.  With trials=False only the
    cache is consulted: on a miss the context's current knobs stay."""
    ctx = ctx or rtseg.default_context(rgbs[0].device.index)
    key = signature(rgbs) + ("" if allow_graph else "|nograph")
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(key)
        except (OSError, ValueError):
            hit = None
        if hit:
            apply(hit["knobs"], ctx)
            return dict(hit, cached=True)
    if not trials:
        return {"knobs": current(ctx), "ms": float("nan"), "seconds": 0.0, "trials": [], "cached": False,
                "source": "current knobs (no cache entry, trials off)"}
    outs = None

    def run():
        nonlocal outs
        outs = rtseg.rt_segment_batch(rgbs, params=params, ctx=ctx)

    best = current(ctx)
    best["graph"] = 0
    apply(best, ctx)
    best_ms = _time(run, reps)
    trials = [(dict(best), best_ms)]
    t0 = time.time()
    for name, values in SPACE.items():
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best, **{name: v})
            apply(cand, ctx)
            ms = _time(run, reps)
            trials.append((cand, ms))
            if verbose:
                print(f"  tune {cand} -> {ms:.3f} ms", flush=True)
            if ms < best_ms:
                best, best_ms = cand, ms
    # graph replay: the first graph holds exactly the rounds the batch needs
    apply(dict(best, recon_round_batch=1), ctx)
    run()
    torch.cuda.synchronize()
    rounds = max(1, rtseg.rt_get_knob("last_rounds", ctx=ctx))
    for budget in (sorted({rounds, rounds + 2}) if allow_graph else []):
        cand = dict(best, graph=1, graph_rounds=budget)
        apply(cand, ctx)
        ms = _time(run, reps)
        trials.append((cand, ms))
        if verbose:
            print(f"  tune {cand} -> {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = cand, ms
    apply(best, ctx)
    res = {"knobs": best, "ms": best_ms, "seconds": round(time.time() - t0, 2),
           "trials": [{"knobs": k, "ms": m} for k, m in trials]}
    if cache:
        try:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = res
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        except (OSError, ValueError):
            pass
    return res
