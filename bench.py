"""Throughput of the plain segmentation pipeline on one MI355X.

One step = rt_segment_tile over one 4096 x 4096 synthetic H&E-like tile (8000
nuclei, semi-axes 4-14 px, 20% in touching clusters of 2-4, jitter +-20,
seed 0), input resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

The roofline object describes the stage that takes the most time, with its
algorithmic bytes per launch (what the launch must read and write at
minimum) divided by its average launch time measured with HIP events that
the library records on its own stream during the timed steps.  The CPU
baseline is the project's oracle (plain single-threaded C) timed on the same
tile on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_4k.json"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU only: tiles are independent, so more GPUs would each run this "
                  "same single-GPU pipeline on their own tiles; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1405_7958_amd import rtseg, synth

    spec = synth.spec_4k(0)
    log(f"generating {spec.w}x{spec.h} tile ...")
    rgb_np, gt, info = synth.make_tile(spec)
    d = torch.device("cuda", 0)
    rgb = torch.from_numpy(rgb_np).to(d)
    ctx = rtseg.Context(0)
    h, w = spec.h, spec.w
    mask = torch.empty((h, w), dtype=torch.uint8, device=d)
    lab = torch.empty((h, w), dtype=torch.int32, device=d)
    n = torch.zeros(1, dtype=torch.int32, device=d)
    out = (mask, lab, n, None)
    params = rtseg.default_params()

    for i in range(args.warmup):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    rtseg.rt_profile_read(ctx)          # discard
    rtseg.rt_profile_enable(True, ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rtseg.rt_profile_enable(False, ctx)
    calls, stages = rtseg.rt_profile_read(ctx)
    n_obj = int(n.item())
    ms_step = (t1 - t0) * 1e3 / args.steps
    tiles_s = args.steps / (t1 - t0)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/tile, {tiles_s:.1f} tiles/s, {n_obj} objects")

    N = w * h
    fg = int((lab > 0).sum().item())
    # algorithmic bytes per launch of each stage (what one launch must move at minimum)
    alg = {
        "deconv": 4 * N,                 # RGB in (3 B/px) + Hq out (1 B/px)
        "level_bound": 2 * N,            # Hq in + lower-bound image out
        "recon": 3 * N,                  # Hq + R in, R out (one full pass)
        "fill_holes": 3 * N,             # Hq + R in, F out
        "ccl": 5 * N,                    # F in, int32 labels out
        "objects": 9 * fg,               # labels in, labels + mask out, on foreground pixels
        "objects_big": 0,
    }
    per_stage = {}
    for k, (ms_tot, launches) in stages.items():
        per_call = ms_tot / max(1, calls)
        per_stage[k] = {"ms_per_tile": round(per_call, 4), "launches_per_tile": round(launches / max(1, calls), 2)}
        log(f"  {k:12s} {per_call:8.4f} ms/tile  launches/tile {launches / max(1, calls):6.2f}")
    dom = max((k for k in stages if alg.get(k, 0) > 0), key=lambda k: stages[k][0])
    ms_tot, launches = stages[dom]
    # one launch processes the whole tile for every stage except recon, whose
    # launches are propagation rounds over active tiles only: count a whole
    # tile pass for the stage
    if dom == "recon":
        t_launch = ms_tot / max(1, calls)
    else:
        t_launch = ms_tot / max(1, launches) * (launches / max(1, calls)) if launches else ms_tot / max(1, calls)
    achieved = alg[dom] / (t_launch * 1e-3) / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("stage") == dom:
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "stage": dom,
            "alg_bytes_per_launch": alg[dom], "ms_per_launch": round(t_launch, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        log("timing the CPU oracle on the same tile (single thread) ...")
        c0 = time.perf_counter()
        hq = oracle.deconv(rgb_np)
        oracle.segment_from_hq(hq)
        c1 = time.perf_counter()
        cpu = {"value": round(1.0 / (c1 - c0), 5), "unit": "tiles/s", "cores": 1, "kind": "oracle",
               "sample": "one full 4096x4096 tile of the same workload (deconvolution + segmentation), "
                         f"single thread, {c1 - c0:.2f} s"}
        log(f"oracle: {c1 - c0:.2f} s/tile")

    line = {
        "metric": "4Kx4K tiles/s on 1 MI355X (plain pipeline); HBM GB/s % of peak",
        "value": round(tiles_s, 3),
        "unit": "tiles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/i32",
        "data": "synthetic",
        "config": {"workload": "plain segmentation pipeline (rt_segment_tile), one 4096x4096 synthetic H&E tile, "
                               "8000 nuclei, semi-axes 4-14 px, 20% in touching clusters of 2-4, jitter +-20, seed 0",
                   "tile": [h, w], "objects": n_obj, "foreground_px": fg,
                   "pipeline_floor_frac": round(8 * N * tiles_s / (HBM_PEAK_GBS * 1e9), 5),
                   "stages": per_stage},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
