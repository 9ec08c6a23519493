#!/usr/bin/env python3
"""Throughput of the Flow Fields hot path on one MI355X.

One step = one ff_flow_fields call on a 1024x436 synthetic pair (the
Sintel-sized plain workload: 16-channel uint8 descriptors, 7x7 SAD patch,
5 scales, 6 propagation steps per scale): descriptors of both images at every
scale, forward and backward fields, both consistency masks.  Inputs are
resident in device memory before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpixel/s fwd+bwd Flow Field at 1024×436 (plain vs learned); EPE on synthetic GT"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pair, c, threads):
    import oracle
    t0 = time.perf_counter()
    oracle.flow_fields(pair.img1, pair.img2, c.levels, c.iters, c.radius, c.R_num, c.R_den, c.eps, c.seed,
                       nthreads=threads)
    dt = time.perf_counter() - t0
    H, W = pair.img1.shape
    return {"value": W * H / dt / 1e6, "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "sample": f"one full {W}x{H} pair (descriptors, fwd+bwd fields, consistency), {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the Flow Fields pair workload is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1703_02563_amd as ff
    from ffgen import CONFIG_PARAMS, epe_stats, make_pair

    cfg = 2
    pair = make_pair(cfg)
    c = CONFIG_PARAMS[cfg]
    H, W = pair.img1.shape
    params = ff.Params(levels=c.levels, iters=c.iters, radius=c.radius, R_num=c.R_num, R_den=c.R_den, eps=c.eps,
                       seed=c.seed)
    dev = torch.device("cuda:0")
    img1 = torch.from_numpy(pair.img1).to(dev)
    img2 = torch.from_numpy(pair.img2).to(dev)
    runner = ff.FlowFields(W, H, params, device=dev)
    log(f"bench: {W}x{H} L={c.levels} T={c.iters}, warmup {args.warmup}")
    for _ in range(args.warmup):
        runner(img1, img2)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runner(img1, img2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = W * H * args.steps / dt / 1e6
    out = runner.out
    n_evals = [int(v) for v in out["n_evals"].cpu()]
    q = epe_stats(out["flow_fwd"].cpu().numpy(), pair.flow_gt, pair.occ, keep=out["keep_fwd"].cpu().numpy())
    log(f"bench: {ms:.3f} ms/step, {value:.1f} Mpix/s, n_evals {n_evals}, quality {q}")

    base = None
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        log(f"bench: CPU oracle baseline on {threads} threads")
        base = cpu_baseline(pair, c, threads)

    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "plain Flow Fields, one 1024x436 uint8 pair (12 polygon layers, t in +-150 px), "
                               "16-ch uint8 descriptors, 7x7 SAD, 5 scales x 6 steps, fwd+bwd+consistency",
                   "W": W, "H": H, "levels": c.levels, "iters": c.iters, "R": f"{c.R_num}/{c.R_den}",
                   "n_evals": n_evals, "epe_raw": round(q["epe"], 4), "le3px": round(q["le3px"], 4),
                   "epe10": round(q["epe10"], 4), "kept_density": round(q["kept_density"], 4),
                   "kept_epe": round(q["kept_epe"], 4)},
        "roofline": None,
        "cpu_baseline": base,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
