"""Throughput of the plain segmentation pipeline on one MI355X.

One step = rt_segment_tile over one 4096 x 4096 synthetic H&E-like tile (8000
nuclei, semi-axes 4-14 px, 20% in touching clusters of 2-4, jitter +-20,
seed 0), input resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-stream4k] [--no-next]
                  [--no-batch] [--no-surrogate] [--no-tune] [--knobs K=V,...]
                  [--copy-calibration MB]

The launch knobs of the 4096 x 4096 tile are picked first by the autotuner
(graph replay excluded, so that stage timing stays available), unless --knobs
gives them (profiler runs pass the set a tuned run reported, so that no
tuning trial enters the kernel statistics).

Roofline: after the timed steps are read, four candidates compete for the
dominant kernel: the reconstruction round kernel and the three per-object
classes (small, medium and large LDS classes, which run side by side on
three streams; the small class is two launches on its stream, a first pass
and the deferred full pass, timed together).  The library records a pair of
HIP events around every launch on the stream the kernel runs on (around each
run of consecutive round launches for the round kernel, around both small
launches) and device counters of the work done.
The kernel with the most time per tile is the dominant one.  Algorithmic
bytes are per call, never per re-visit: the uint8 reconstruction moves 3 B
per pixel of the tile per call (read Hq and R, write R), spread over the
call's round launches; a per-object kernel moves 9 B per pixel of the
components it processes (read the label, write label and mask).  `value`
comes from the same timed steps (the events add no synchronisation).
`pipeline_floor_frac` is the whole tile's 8 B/px floor (RGB in, mask and
labels out) at the measured tiles/s, as a fraction of the 8 TB/s peak.

The "next_rows" object times the stages built beside the segmentation on the
same tile: rt_features, rt_morph (opening), rt_recon_to_nuclei (opening by
reconstruction), rt_rbc_detect and rt_segment_slide (stitching).  The
"host_stream4k" object times rt_segment_host_stream over the distinct tiles
below held in pinned host memory (every copy inside the timed region), with
the copies overlapped (depth 3) and not (depth 1).

The "stream4k" object times rt_segment_batch over 8 distinct 4096 x 4096
tiles of the same generator (seeds 0..7) per call: every tile's data is
different, so the 1.2 GB working set cannot stay in the 256 MB MALL between
steps.

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

The CPU baseline is the project's oracle (plain single-threaded C, the same
source built -O3 -march=native -ffp-contract=off on this host) timed on the
same 4096 x 4096 tile: once on one core, then one copy of the tile per
available core in as many threads (tile-parallel); `value` is the all-core
tiles/s.

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
BF16_PEAK_TFLOPS = 2500.0
METRIC = "4K\u00d74K tiles/s on 1 MI355X: plain vs surrogate @Dice\u22650.95; HBM GB/s % of peak"
ROUND_KERNEL = "k_recon_round<unsigned char, 8, true>"   # the plain uint8 round kernel
# the small class runs as two launches on its stream (first pass, then the
# deferred full pass); one event pair spans both
OBJ_KERNELS = ("k_objects_s1+k_objects_s", "k_objects_m", "k_objects_l")
OBJ_BYTES_PER_PX = 9      # read the label, write label (4 B) and mask (1 B)
RECON_BYTES_PER_PX = 3    # uint8 reconstruction per call: read Hq and R, write R


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
    res = tune.autotune(rgbs, ctx=ctx, reps=3, cache=tune_cache(args), trials=args.tune_trials)
    log(f"{'cached' if res.get('cached') else 'tuner'} knobs {res['knobs']} ({res['ms']:.2f} ms/batch)")
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
           "objects": objs, "knobs": res["knobs"],
           "knobs_source": "tune cache" if res.get("cached") else res.get("source", "autotuned"),
           "pipeline_floor_frac": round(8 * px / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 5)}
    ctx.close()
    return out


def distinct_4k_tiles(synth, torch, n):
    """n distinct 4096 x 4096 tiles of the 4096 x 4096 workload's generator
    (seeds 0..n-1), as pinned host tensors."""
    from concurrent.futures import ThreadPoolExecutor
    base = synth.spec_4k(0)
    specs = [synth.TileSpec(w=base.w, h=base.h, seed=i, n_nuclei=base.n_nuclei, amin=base.amin, amax=base.amax,
                            cluster_frac=base.cluster_frac, cluster_min=base.cluster_min, cluster_max=base.cluster_max,
                            jitter=base.jitter) for i in range(n)]
    log(f"generating {n} distinct 4096x4096 tiles ...")
    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(lambda s: torch.from_numpy(synth.make_tile(s)[0]).pin_memory(), specs))


def stream4k(rtseg, synth, torch, args, knobs, host_tiles):
    """rt_segment_batch over `args.stream4k_tiles` distinct 4096 x 4096 tiles
    (the 4096 x 4096 workload's generator, seeds 0..n-1) per call, with the
    knob set of the single 4096 x 4096 tile (no tuning trials)."""
    from paper_1405_7958_amd import tune
    d = torch.device("cuda", 0)
    nt = len(host_tiles)
    base = synth.spec_4k(0)
    rgbs = [t.to(d) for t in host_tiles]
    ctx = rtseg.Context(0)
    if knobs:
        tune.apply(knobs, ctx)
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
    ms = (t1 - t0) * 1e3 / steps
    px = nt * base.w * base.h
    tps = nt / (ms * 1e-3)
    objs = sum(int(o[2].item()) for o in outs)
    log(f"stream4k: {ms:.2f} ms per {nt} tiles, {tps:.1f} tiles/s")
    out = {"tiles_per_call": nt, "seeds": [0, nt - 1], "steps": steps, "ms_per_call": round(ms, 3),
           "tiles_per_s": round(tps, 2), "mpx_per_s": round(px / (ms * 1e-3) / 1e6, 1), "objects": objs,
           "working_set_mb": round(nt * base.w * base.h * (3 + 1 + 4) / 1e6, 1),
           "knobs": knobs, "knobs_source": "the 4096x4096 tile's knob set" if knobs else "defaults",
           "pipeline_floor_frac": round(8 * px / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 5)}
    ctx.close()
    return out


def host_stream_leg(rtseg, torch, knobs, host_tiles, reps=2):
    """rt_segment_host_stream over the distinct 4096 x 4096 tiles held in
    pinned host memory: uploads (RGB), computation and downloads (mask,
    labels, count) overlapped (depth 3) against one after the other (depth 1);
    tiles/s with every host-device copy inside the timed region."""
    from paper_1405_7958_amd import tune
    ctx = rtseg.Context(0)
    if knobs:
        tune.apply(knobs, ctx)
    n = len(host_tiles)
    out = {"tiles_per_call": n, "reps": reps}
    outs = None
    for depth in (3, 1):
        outs = rtseg.rt_segment_host_stream(host_tiles, depth=depth, ctx=ctx, outs=outs)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rtseg.rt_segment_host_stream(host_tiles, depth=depth, ctx=ctx, outs=outs)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        out[f"depth{depth}_tiles_per_s"] = round(n / sec, 2)
        out[f"depth{depth}_ms_per_tile"] = round(sec * 1e3 / n, 3)
        log(f"host stream depth {depth}: {n / sec:.1f} tiles/s ({sec * 1e3 / n:.2f} ms/tile, copies included)")
    px = host_tiles[0].shape[0] * host_tiles[0].shape[1]
    out["pcie_bytes_per_tile"] = px * (3 + 1 + 4) + 4
    out["overlap_gain"] = round(out["depth3_tiles_per_s"] / out["depth1_tiles_per_s"], 3)
    out["pcie_gbs_depth3"] = round(out["pcie_bytes_per_tile"] * out["depth3_tiles_per_s"] / 1e9, 2)
    ctx.close()
    return out


def next_rows_leg(rtseg, torch, rgb, lab, ctx, reps=5):
    """The stages built beside the segmentation, timed on the 4096 x 4096
    tile (device-resident): feature computation on the segmentation's labels,
    disk opening, ReconToNuclei with the opening-by-reconstruction marker,
    RBC detection, and cross-tile stitching (1024 x 1024 cores, 64-px halo)."""
    hq = rtseg.rt_deconv(rgb, ctx=ctx)
    H, W = hq.shape
    N = H * W

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out = {}
    nuc = {}

    def feats():
        nuc["n"] = rtseg.rt_features(lab, hq, max_nuclei=16384, ctx=ctx)[3]
    ms = timed(feats)
    out["features"] = {"ms_per_tile": round(ms, 3), "nuclei": nuc["n"], "nuclei_per_s": round(nuc["n"] / ms * 1e3),
                       "read_gbs": round(5 * N / (ms * 1e-3) / 1e9, 1),
                       "note": "includes one count read-back per call (binding)"}
    ms = timed(lambda: rtseg.rt_morph(hq, rtseg.RT_OPEN, 5, ctx=ctx))
    out["morph_open_r5"] = {"ms_per_tile": round(ms, 3), "gbs": round(4 * N / (ms * 1e-3) / 1e9, 1)}
    ms = timed(lambda: rtseg.rt_recon_to_nuclei(hq, rtseg.RT_MARKER_OPEN, 5, 16, ctx=ctx))
    out["recon_to_nuclei_open_r5"] = {"ms_per_tile": round(ms, 3)}
    ms = timed(lambda: rtseg.rt_rbc_detect(rgb, 200, 150, ctx=ctx))
    out["rbc_detect"] = {"ms_per_tile": round(ms, 3)}
    ms = timed(lambda: rtseg.rt_segment_slide(rgb, 1024, 64, ctx=ctx))
    out["stitch_1024_halo64"] = {"ms_per_slide": round(ms, 3), "mpx_per_s": round(N / (ms * 1e-3) / 1e6, 1),
                                 "cores": 16}
    for k, v in out.items():
        log(f"  {k:28s} {v}")
    return out


def unet_forward_flops_per_px():
    """Algorithmic FLOPs per input pixel of one U-Net forward pass (2 per
    multiply-add; RGB input, levels of 16/32/64/128 channels, two 3x3 convs
    per level, 2x2 stride-2 up-convs, 1x1 head to 2 maps)."""
    ch = (16, 32, 64, 128)
    f = 0.0
    cin = 3
    for lvl, c in enumerate(ch):              # encoder and bottleneck
        f += 2 * 9 * (cin * c + c * c) / 4 ** lvl
        cin = c
    for lvl in (2, 1, 0):                     # decoder
        c = ch[lvl]
        f += 2 * ch[lvl + 1] * c / 4 ** lvl   # up-conv: one input pixel per output pixel
        f += 2 * 9 * (2 * c * c + c * c) / 4 ** lvl
    return f + 2 * ch[0] * 2


def surrogate_forward_rate(rtseg, torch, net, tile, reps=5):
    """Times rt_unet_forward on one tile; FLOPs counted over the inference
    windows (512 x 512 at stride 480, the last flush with the edge)."""
    h, w = tile.shape[:2]

    def nwin(n):
        return 1 if n <= 512 else 1 + -(-(n - 512) // 480)
    px = nwin(h) * nwin(w) * 512 * 512
    net.forward(tile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(tile)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = unet_forward_flops_per_px() * px
    tf = flops / (ms * 1e-3) / 1e12
    return {"ms_per_tile": round(ms, 3), "tflop_per_tile": round(flops / 1e12, 4), "achieved_tflops": round(tf, 1),
            "peak_tflops": BF16_PEAK_TFLOPS, "mfma_frac": round(tf / BF16_PEAK_TFLOPS, 5), "window_px": px}


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
    fwd = surrogate_forward_rate(rtseg, torch, net, held[0])
    log(f"U-Net forward on a 4096x4096 tile: {fwd['ms_per_tile']} ms, {fwd['achieved_tflops']} TFLOP/s "
        f"({fwd['mfma_frac']:.4f} of the bf16 MFMA peak)")
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
        return {"weights": src, "training": train, "forward": fwd, "heldout_4k": cfg4, "stream": None}
    # config 5: a sample of the mixed stream, surrogate + fallback
    from concurrent.futures import ThreadPoolExecutor
    specs = [synth.spec_stream(20000 + i) for i in range(args.stream)]
    tiles = []
    with ThreadPoolExecutor(8) as ex:
        for k0 in range(0, len(specs), 64):   # a progress line per 64 tiles
            tiles += list(ex.map(lambda s: torch.from_numpy(synth.make_tile(s)[0]).to(d), specs[k0:k0 + 64]))
            log(f"stream tiles generated: {len(tiles)}/{len(specs)}")
    recs, t_plain, t_sur = surrogate.evaluate(net, tiles, tau=args.tau, ctx=ctx)
    dice = np.array([1.0 if r["fallback"] else r["dice"] for r in recs])
    raw = np.array([r["dice"] for r in recs])
    fb = np.array([r["fallback"] for r in recs])
    px = sum(s.w * s.h for s in specs)
    cfg5 = {"tiles": len(tiles), "of_stream_tiles": 1024,
            "sample": f"the first {len(tiles)} tiles (seeds 20000..{20000 + len(tiles) - 1}) of the 1,024-tile mixed "
                      "stream" if len(tiles) < 1024 else "the whole 1,024-tile mixed stream",
            "megapixels": round(px / 1e6, 1), "tau": args.tau,
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
    return {"weights": src, "training": train, "forward": fwd, "heldout_4k": cfg4, "stream": cfg5}


def cpu_baseline(rgb_np):
    """The oracle on this host's cores: one tile on one core, then one copy of
    the tile per available core, one thread each (the C calls release the
    interpreter lock, so the threads run in parallel)."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    oracle.use_library(oracle.build_native(tmp))

    def one(_):
        oracle.segment_from_hq(oracle.deconv(rgb_np))

    log("timing the CPU oracle on the 4096x4096 tile: one core ...")
    c0 = time.perf_counter()
    one(0)
    t1 = time.perf_counter() - c0
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cores = os.cpu_count() or 1
    log(f"oracle: {t1:.2f} s/tile on one core; {cores} tiles on {cores} threads ...")
    c0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(cores)))
    tall = time.perf_counter() - c0
    log(f"oracle: {cores} tiles in {tall:.2f} s")
    return {"value": round(cores / tall, 5), "unit": "tiles/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} copies of the 4096x4096 tile (deconvolution + segmentation), one per thread, "
                      f"{tall:.2f} s wall; single core: one tile in {t1:.2f} s",
            "single_core_value": round(1.0 / t1, 5),
            "build": "gcc -O3 -march=native -ffp-contract=off (built on this host)", "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_4k.json"))
    ap.add_argument("--no-stream4k", action="store_true")
    ap.add_argument("--no-next", action="store_true", help="skip the stages beside the segmentation")
    ap.add_argument("--tune-trials", action="store_true",
                    help="run tuning trials on a cache miss (default: the cached knob set or the defaults)")
    ap.add_argument("--stream4k-tiles", type=int, default=8)
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
        res = tune.autotune([rgb], ctx=ctx, reps=3, cache=tune_cache(args), allow_graph=False,
                            trials=args.tune_trials)
        knobs = res["knobs"]
        knobs_source = "tune cache" if res.get("cached") else res.get("source", "autotuned")
        log(f"{knobs_source} knobs for the 4096x4096 tile: {knobs} ({res['ms']:.3f} ms, {res['seconds']} s)")
    for i in range(args.warmup):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    # the timed steps record the candidate kernels' timing: HIP events around
    # each run of round launches and around each per-object class launch, on
    # the stream each runs on, plus device counters of the work done
    rtseg.rt_profile_enable(2, ctx)
    rtseg.rt_profile_recon_rounds(ctx)  # discard
    for k in range(3):
        rtseg.rt_profile_objects(k, ctx)  # discard
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r_ms, r_launches, r_visits = rtseg.rt_profile_recon_rounds(ctx)
    obj = [rtseg.rt_profile_objects(k, ctx) for k in range(3)]
    rtseg.rt_profile_enable(False, ctx)
    n_obj = int(n.item())
    ms_step = (t1 - t0) * 1e3 / args.steps
    tiles_s = args.steps / (t1 - t0)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/tile, {tiles_s:.1f} tiles/s, {n_obj} objects")
    # ... then the same steps again with HIP events at every stage boundary
    rtseg.rt_profile_enable(True, ctx)
    rtseg.rt_profile_read(ctx)          # discard
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(args.steps):
        rtseg.rt_segment_tile(rgb, params, ctx=ctx, out=out)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rtseg.rt_profile_enable(False, ctx)
    calls, stages = rtseg.rt_profile_read(ctx)
    rtseg.rt_profile_recon_rounds(ctx)  # the timed steps' figures are kept
    for k in range(3):
        rtseg.rt_profile_objects(k, ctx)
    ms_prof = (t3 - t2) * 1e3 / args.steps
    log(f"instrumented steps: {ms_prof:.3f} ms/tile")

    N = w * h
    fg = int((lab > 0).sum().item())
    per_stage = {}
    for k, (ms_tot, launches) in stages.items():
        per_call = ms_tot / max(1, calls)
        per_stage[k] = {"ms_per_tile": round(per_call, 4), "launches_per_tile": round(launches / max(1, calls), 2)}
        log(f"  {k:12s} {per_call:8.4f} ms/tile  launches/tile {launches / max(1, calls):6.2f}")
    # candidate kernels: time per tile, algorithmic bytes per launch, rate
    kern = []
    if r_launches:
        kern.append({"kernel": ROUND_KERNEL, "ms_per_tile": r_ms / args.steps, "launches": r_launches,
                     "us_per_launch": r_ms * 1e3 / r_launches,
                     "alg_bytes_per_launch": RECON_BYTES_PER_PX * N * args.steps / r_launches,
                     "alg_bytes_rule": "3 B per tile pixel per call (read Hq and R, write R), over the call's "
                                       "round launches",
                     "tile_visits_per_launch": round(r_visits / r_launches, 1)})
    for name, (ms_k, ln_k, px_k) in zip(OBJ_KERNELS, obj):
        if ln_k:
            kern.append({"kernel": name, "ms_per_tile": ms_k / args.steps, "launches": ln_k,
                         "us_per_launch": ms_k * 1e3 / ln_k, "alg_bytes_per_launch": OBJ_BYTES_PER_PX * px_k / ln_k,
                         "alg_bytes_rule": "9 B per pixel of the components the class processed (device count)",
                         "component_px_per_launch": round(px_k / ln_k)})
    for k in kern:
        k["achieved_gbs"] = k["alg_bytes_per_launch"] / (k["us_per_launch"] * 1e-6) / 1e9
        k["frac"] = k["achieved_gbs"] / HBM_PEAK_GBS
        log(f"  {k['kernel']:40s} {k['ms_per_tile'] * 1e3:8.1f} us/tile {k['us_per_launch']:8.1f} us/launch "
            f"{k['alg_bytes_per_launch'] / 1e6:8.2f} MB/launch {k['achieved_gbs']:8.1f} GB/s")
    dom = max(kern, key=lambda k: k["ms_per_tile"])
    # counter traffic of the dominant kernel (two rocprofv3 --pmc runs,
    # calibrated by a copy), valid for the knob set the counters were taken with
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            used = knobs or {k: rtseg.rt_get_knob(k, ctx=ctx) for k in rtseg.KNOBS}
            same = all(int(used.get(k, -1)) == int(v) for k, v in tj.get("knobs", {}).items()
                       if k in ("recon_levels", "recon_level_mode", "recon_level_frac", "recon_round_batch"))
            traffic = tj.get("bytes_per_launch", {}).get(dom["kernel"]) if same and tj.get("knobs") else None
        except Exception:
            traffic = None
    floor_frac = 8 * N * tiles_s / (HBM_PEAK_GBS * 1e9)
    roof = {"bound": "hbm", "achieved": round(dom["achieved_gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom["frac"], 5), "traffic": traffic, "kernel": dom["kernel"],
            "alg_bytes_per_launch": round(dom["alg_bytes_per_launch"]), "us_per_launch": round(dom["us_per_launch"], 2),
            "pipeline_floor_frac": round(floor_frac, 5),
            "kernels": [{k2: (round(v, 5) if isinstance(v, float) else v) for k2, v in k.items()} for k in kern]}

    nxt = None
    if not args.no_next:
        log("stages beside the segmentation on the 4096x4096 tile:")
        nxt = next_rows_leg(rtseg, torch, rgb, lab, ctx)
    batch = None
    if not args.no_batch:
        batch = batch64(rtseg, synth, torch, args)
    s4k = hs = None
    if not args.no_stream4k:
        host_tiles = distinct_4k_tiles(synth, torch, args.stream4k_tiles)
        s4k = stream4k(rtseg, synth, torch, args, knobs, host_tiles)
        hs = host_stream_leg(rtseg, torch, knobs, host_tiles)
        del host_tiles
    sur = None
    if not args.no_surrogate:
        sur = surrogate_leg(rtseg, synth, torch, args, ms_step)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(rgb_np)

    line = {
        "metric": METRIC,
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
                   "pipeline_floor_frac": round(floor_frac, 5),
                   "knobs": knobs, "knobs_source": knobs_source, "ms_per_step_instrumented": round(ms_prof, 4), "stages": per_stage},
        "roofline": roof,
        "batch64": batch,
        "next_rows": nxt,
        "stream4k": s4k,
        "host_stream4k": hs,
        "surrogate": sur,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
