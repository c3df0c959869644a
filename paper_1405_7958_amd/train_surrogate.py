"""Trains the U-Net surrogate on crops labelled by the plain pipeline.

  python -m paper_1405_7958_amd.train_surrogate --crops 2000 --epochs 4 \
      --out weights.bin [--log-json curve.json] [--time-budget S]

Crops: 512 x 512 from tiles of the mixed stream (seeds from 10000 on), each
tile segmented whole by the plain pipeline; targets are its foreground after
the first area threshold and its dilated watershed seeds.  Every network
step runs in the library's kernels.  Prints progress to stderr and a JSON
summary line to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--crops", type=int, default=2000)
    ap.add_argument("--epochs", type=float, default=4.0)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--w-seed", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-budget", type=float, default=None)
    ap.add_argument("--out", required=True)
    ap.add_argument("--log-json", default=None)
    args = ap.parse_args()

    import torch
    from paper_1405_7958_amd import rtseg, surrogate

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    d = torch.device("cuda", 0)
    ctx = rtseg.Context(0)
    t0 = time.time()
    data = surrogate.make_training_set(args.crops, device=d, ctx=ctx, log=log)
    t_data = time.time() - t0
    fg_frac = float(data[1].float().mean().item())
    sd_frac = float(data[2].float().mean().item())
    log(f"data: {args.crops} crops in {t_data:.1f} s, fg {fg_frac:.3f}, seeds {sd_frac:.4f}")
    net = rtseg.UNet(seed=args.seed, ctx=ctx)
    losses, secs, steps = surrogate.train(net, data, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                         w_seed=args.w_seed, log=log, time_budget=args.time_budget)
    net.save(args.out)
    px = steps * args.batch * 512 * 512
    summary = {"crops": args.crops, "epochs": args.epochs, "batch": args.batch, "steps": steps,
               "train_seconds": round(secs, 2), "data_seconds": round(t_data, 2),
               "train_mpx_per_s": round(px / secs / 1e6, 2),
               "train_tflops": round(3 * 70.8e3 * px / secs / 1e12, 2),
               "loss_first": losses[0], "loss_last": sum(losses[-20:]) / len(losses[-20:]),
               "fg_fraction": fg_frac, "seed_fraction": sd_frac, "weights": args.out}
    if args.log_json:
        with open(args.log_json, "w") as f:
            json.dump(dict(summary, losses=losses), f)
    print(json.dumps(summary), flush=True)
    net.close()


if __name__ == "__main__":
    main()
