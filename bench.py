"""Throughput of the plain segmentation pipeline on one MI355X.

One step = rt_segment_tile over one 4096 x 4096 synthetic H&E-like tile (8000
nuclei, semi-axes 4-14 px, 20% in touching clusters of 2-4, jitter +-20,
seed 0), input resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                  [--no-batch] [--no-surrogate] [--no-tune] [--knobs K=V,...]
                  [--copy-calibration MB]

The launch knobs of the 4096 x 4096 tile are picked first by the autotuner
(graph replay excluded, so that stage timing stays available), unless --knobs
gives them (profiler runs pass the set a tuned run reported, so that no
tuning trial enters the kernel statistics).

Roofline: the dominant kernel is the reconstruction round kernel (most of the
GPU time of a tile).  After the timed steps, the same number of steps runs
again with the library's stage timing on: HIP events at every stage boundary
and a pair around every round launch, on the call's stream, plus a count of
the 62 x 62 tiles the rounds process; achieved = tile visits x 11532
algorithmic bytes (read Hq and R, write R: 3 bytes per interior pixel) /
summed kernel time.  `value` comes from the uninstrumented steps.

The "batch64" object times rt_segment_batch on the 64-tile batch of uneven
slide-edge sizes (each side drawn from {512, 1024, 2048, 4096}), with knobs
picked by the autotuner on that batch.

The "surrogate" object compares the U-Net surrogate (rt_segment_tile_surrogate)
with the plain pipeline: on held-out 4096 x 4096 tiles without fallback (Dice,
IoU, tiles/s) and on a sample of the mixed stream (60% normal, 30% dense, 10%
low contrast; sizes 512..4096 per side) with plain fallback below confidence
tau (tiles/s of both, fallback rate, Dice with fallback tiles counting 1).
Weights come from --weights if that file exists, else the network is trained
in the run on --train-crops crops labelled by the plain pipeline.

The CPU baseline is the project's oracle (plain single-threaded C) timed on
the same 4096 x 4096 tile on this host.

--copy-calibration MB runs one plain device copy of MB MiB before anything
else, so that a counter run (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE) sees a
kernel of known traffic beside the pipeline kernels.
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
TILE_VISIT_BYTES = 62 * 62 * 3
ROUND_KERNEL = "k_recon_round<unsigned char, 8, true>"   # the plain uint8 round kernel


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 0
    return f"{model}, {n} cores available"


def tune_cache(args):
    return None if args.tune_cache.lower() == "none" else args.tune_cache


def batch64(rtseg, synth, torch, args):
    from concurrent.futures import ThreadPoolExecutor

    from paper_1405_7958_amd import tune
    d = torch.device("cuda", 0)
    specs = [synth.spec_uneven(i) for i in range(64)]
    log("generating the 64-tile uneven batch ...")
    with ThreadPoolExecutor(8) as ex:
        rgbs = list(ex.map(lambda s: torch.from_numpy(synth.make_tile(s)[0]).to(d), specs))
    ctx = rtseg.Context(0)
    res = tune.autotune(rgbs, ctx=ctx, reps=3, cache=tune_cache(args))
    log(f"{'cached' if res.get('cached') else 'autotuned'} knobs {res['knobs']} ({res['ms']:.2f} ms/batch, "
        f"{res['seconds']} s)")
    params = rtseg.default_params()
    for _ in range(2):
        rtseg.rt_segment_batch(rgbs, params, ctx=ctx)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        outs = rtseg.rt_segment_batch(rgbs, params, ctx=ctx)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    px = sum(s.w * s.h for s in specs)
    ms = (t1 - t0) * 1e3 / steps
    objs = sum(int(o[2].item()) for o in outs)
    log(f"batch64: {ms:.2f} ms/batch, {64 / (ms * 1e-3):.1f} tiles/s, {px / (ms * 1e-3) / 1e6:.0f} Mpx/s")
    out = {"tiles": 64, "megapixels": round(px / 1e6, 2), "steps": steps, "ms_per_batch": round(ms, 3),
           "tiles_per_s": round(64 / (ms * 1e-3), 2), "mpx_per_s": round(px / (ms * 1e-3) / 1e6, 1),
           "objects": objs, "knobs": res["knobs"], "knobs_source": "tune cache" if res.get("cached") else "autotuned",
           "pipeline_floor_frac": round(8 * px / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 5)}
    ctx.close()
    return out


def surrogate_leg(rtseg, synth, torch, args, plain_ms_4k):
    """Configs 4/5: the U-Net surrogate (+ plain fallback) against the plain
    pipeline: 4096 x 4096 held-out tiles (Dice / IoU, tiles/s) and a sample
    of the mixed stream (tiles/s of both, fallback rate, Dice)."""
    import numpy as np

    from paper_1405_7958_amd import surrogate
    d = torch.device("cuda", 0)
    ctx = rtseg.Context(0)
    net = rtseg.UNet(seed=0, ctx=ctx)
    train = None
    if args.weights and os.path.exists(args.weights):
        net.load(args.weights)
        src = os.path.relpath(args.weights, ROOT)
        log(f"surrogate weights loaded from {src}")
    else:
        log(f"training the surrogate: {args.train_crops} crops, {args.train_epochs} epochs ...")
        t0 = time.time()
        data = surrogate.make_training_set(args.train_crops, device=d, ctx=ctx)
        t_data = time.time() - t0
        losses, secs, steps = surrogate.train(net, data, epochs=args.train_epochs, batch=8, lr=2e-3, log=log)
        px = steps * 8 * 512 * 512
        train = {"crops": args.train_crops, "epochs": args.train_epochs, "steps": steps, "seconds": round(secs, 2),
                 "data_seconds": round(t_data, 1), "mpx_per_s": round(px / secs / 1e6, 1),
                 "loss_first": round(losses[0], 4), "loss_last": round(float(np.mean(losses[-10:])), 4)}
        src = "trained in this run"
        del data
    # config 4: held-out 4096 x 4096 tiles, surrogate alone (no fallback)
    held = []
    for i in range(args.heldout):
        spec = synth.spec_4k(0)
        spec = synth.TileSpec(w=4096, h=4096, seed=15000 + i, n_nuclei=spec.n_nuclei, amin=spec.amin, amax=spec.amax,
                              cluster_frac=spec.cluster_frac, cluster_min=spec.cluster_min,
                              cluster_max=spec.cluster_max, jitter=spec.jitter)
        held.append(torch.from_numpy(synth.make_tile(spec)[0]).to(d))
    for t in held[:1]:   # warm-up
        rtseg.rt_segment_tile_surrogate(t, net, tau=-1.0, ctx=ctx)
    recs, t_plain, t_sur = surrogate.evaluate(net, held, tau=-1.0, ctx=ctx)
    dice = [r["dice"] for r in recs]
    iou = [r["iou"] for r in recs]
    cfg4 = {"tiles": len(held), "tile": [4096, 4096], "surrogate_tiles_per_s": round(len(held) / t_sur, 2),
            "plain_tiles_per_s": round(len(held) / t_plain, 2), "dice_mean": round(float(np.mean(dice)), 4),
            "iou_mean": round(float(np.mean(iou)), 4), "confidence": [round(r["confidence"], 3) for r in recs]}
    log(f"held-out 4K: surrogate {cfg4['surrogate_tiles_per_s']} tiles/s, plain {cfg4['plain_tiles_per_s']} "
        f"tiles/s, Dice {cfg4['dice_mean']}, IoU {cfg4['iou_mean']}")
    if args.stream <= 0:
        net.close()
        ctx.close()
        return {"weights": src, "training": train, "heldout_4k": cfg4, "stream": None}
    # config 5: a sample of the mixed stream, surrogate + fallback
    from concurrent.futures import ThreadPoolExecutor
    specs = [synth.spec_stream(20000 + i) for i in range(args.stream)]
    with ThreadPoolExecutor(8) as ex:
        tiles = list(ex.map(lambda s: torch.from_numpy(synth.make_tile(s)[0]).to(d), specs))
    recs, t_plain, t_sur = surrogate.evaluate(net, tiles, tau=args.tau, ctx=ctx)
    dice = np.array([1.0 if r["fallback"] else r["dice"] for r in recs])
    raw = np.array([r["dice"] for r in recs])
    fb = np.array([r["fallback"] for r in recs])
    px = sum(s.w * s.h for s in specs)
    cfg5 = {"tiles": len(tiles), "megapixels": round(px / 1e6, 1), "tau": args.tau,
            "surrogate_tiles_per_s": round(len(tiles) / t_sur, 2), "plain_tiles_per_s": round(len(tiles) / t_plain, 2),
            "fallback_rate": round(float(fb.mean()), 4), "dice_mean": round(float(dice.mean()), 4),
            "dice_p5": round(float(np.percentile(dice, 5)), 4),
            "dice_surrogate_tiles_mean": round(float(raw[~fb].mean()), 4) if (~fb).any() else None,
            "by_kind": {k: round(float(dice[[s.kind == k for s in specs]].mean()), 4)
                        for k in ("normal", "dense", "low_contrast") if any(s.kind == k for s in specs)},
            "per_tile": [[s.kind[0], round(r["confidence"], 3), round(r["dice"], 4)] for s, r in zip(specs, recs)]}
    log(f"stream sample: surrogate+fallback {cfg5['surrogate_tiles_per_s']} tiles/s, plain "
        f"{cfg5['plain_tiles_per_s']} tiles/s, fallback {cfg5['fallback_rate']}, Dice {cfg5['dice_mean']} "
        f"(p5 {cfg5['dice_p5']})")
    net.close()
    ctx.close()
    return {"weights": src, "training": train, "heldout_4k": cfg4, "stream": cfg5}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_recon_round_4k.json"))
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default knobs for the 4096x4096 tile")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1405_7958_amd", "tune_cache.json"),
                    help="autotuner cache (knob sets by device and tile sizes); 'none' tunes afresh")
    ap.add_argument("--knobs", default="", metavar="K=V,...",
                    help="knobs for the 4096x4096 tile instead of autotuning (e.g. the set a tuned run reported)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1405_7958_amd", "weights", "unet_surrogate.rtunet"))
    ap.add_argument("--train-crops", type=int, default=512)
    ap.add_argument("--train-epochs", type=float, default=2.0)
    ap.add_argument("--heldout", type=int, default=2)
    ap.add_argument("--stream", type=int, default=48)
    ap.add_argument("--tau", type=float, default=0.8)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU only: tiles are independent, so more GPUs would each run this "
                  "same single-GPU pipeline on their own tiles; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1405_7958_amd import rtseg, synth

    d = torch.device("cuda", 0)
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb, dtype=torch.uint8, device=d)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_calibration} MiB done")
        del src, dst

    spec = synth.spec_4k(0)
    log(f"generating {spec.w}x{spec.h} tile ...")
    rgb_np, gt, info = synth.make_tile(spec)
    rgb = torch.from_numpy(rgb_np).to(d)
    ctx = rtseg.Context(0)
    h, w = spec.h, spec.w
    mask = torch.empty((h, w), dtype=torch.uint8, device=d)
    lab = torch.empty((h, w), dtype=torch.int32, device=d)
    n = torch.zeros(1, dtype=torch.int32, device=d)
    out = (mask, lab, n, None)
    params = rtseg.default_params()

    knobs = None
    knobs_source = "defaults"
    if args.knobs:
        knobs_source = "--knobs"
        knobs = {}
        for kv in args.knobs.split(","):
            k, v = kv.split("=")
            rtseg.rt_set_knob(k.strip(), int(v), ctx=ctx)
            knobs[k.strip()] = int(v)
        log(f"knobs for the 4096x4096 tile: {knobs}")
    elif not args.no_tune:
        from paper_1405_7958_amd import tune
        res = tune.autotune([rgb], ctx=ctx, reps=3, cache=tune_cache(args), allow_graph=False)
        knobs = res["knobs"]
        knobs_source = "tune cache" if res.get("cached") else "autotuned"
        log(f"{knobs_source} knobs for the 4096x4096 tile: {knobs} ({res['ms']:.3f} ms, {res['seconds']} s)")
    for i in range(args.warmup):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    # the timed steps record only the round kernel's timing (two HIP events
    # around each run of round launches on the call's stream, and the number
    # of tiles each launch processes) ...
    rtseg.rt_profile_enable(2, ctx)
    rtseg.rt_profile_recon_rounds(ctx)  # discard
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r_ms, r_launches, r_visits = rtseg.rt_profile_recon_rounds(ctx)
    rtseg.rt_profile_enable(False, ctx)
    n_obj = int(n.item())
    ms_step = (t1 - t0) * 1e3 / args.steps
    tiles_s = args.steps / (t1 - t0)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/tile, {tiles_s:.1f} tiles/s, {n_obj} objects")
    # ... then the same steps again with HIP events at every stage boundary
    rtseg.rt_profile_enable(True, ctx)
    rtseg.rt_profile_read(ctx)          # discard
    rtseg.rt_profile_recon_rounds(ctx)  # discard
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(args.steps):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rtseg.rt_profile_enable(False, ctx)
    calls, stages = rtseg.rt_profile_read(ctx)
    rtseg.rt_profile_recon_rounds(ctx)  # the timed steps' figures are kept
    ms_prof = (t3 - t2) * 1e3 / args.steps
    log(f"instrumented steps: {ms_prof:.3f} ms/tile")

    N = w * h
    fg = int((lab > 0).sum().item())
    per_stage = {}
    for k, (ms_tot, launches) in stages.items():
        per_call = ms_tot / max(1, calls)
        per_stage[k] = {"ms_per_tile": round(per_call, 4), "launches_per_tile": round(launches / max(1, calls), 2)}
        log(f"  {k:12s} {per_call:8.4f} ms/tile  launches/tile {launches / max(1, calls):6.2f}")
    # dominant kernel: the reconstruction round kernel
    ms_launch = r_ms / max(1, r_launches)
    bytes_launch = TILE_VISIT_BYTES * r_visits / max(1, r_launches)
    achieved = bytes_launch / (ms_launch * 1e-3) / 1e9 if r_launches else 0.0
    log(f"recon round kernel: {r_launches} launches, {ms_launch * 1e3:.1f} us/launch, "
        f"{r_visits / max(1, r_launches):.0f} tile visits/launch, {achieved:.1f} GB/s")
    # counter traffic of the round kernel, measured for one knob set: it holds
    # for this run when the knobs that change a launch's work agree
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            used = knobs or {k: rtseg.rt_get_knob(k, ctx=ctx) for k in rtseg.KNOBS}
            same = all(int(used.get(k, -1)) == int(v) for k, v in tj.get("knobs", {}).items()
                       if k in ("recon_levels", "recon_level_mode", "recon_level_frac", "recon_round_batch"))
            same = same and tj.get("kernel") == ROUND_KERNEL   # counters of this kernel's code
            traffic = tj.get("bytes_per_launch") if same and tj.get("knobs") else None
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "kernel": ROUND_KERNEL,
            "alg_bytes_per_launch": round(bytes_launch), "us_per_launch": round(ms_launch * 1e3, 2),
            "launches_per_tile": round(r_launches / max(1, args.steps), 2),
            "tile_visits_per_launch": round(r_visits / max(1, r_launches), 1)}

    batch = None
    if not args.no_batch:
        batch = batch64(rtseg, synth, torch, args)
    sur = None
    if not args.no_surrogate:
        sur = surrogate_leg(rtseg, synth, torch, args, ms_step)

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
                         f"single thread, {c1 - c0:.2f} s",
               "host": host_cpu()}
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
                   "knobs": knobs, "knobs_source": knobs_source, "ms_per_step_instrumented": round(ms_prof, 4), "stages": per_stage},
        "roofline": roof,
        "batch64": batch,
        "surrogate": sur,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
