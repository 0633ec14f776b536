"""Throughput of the decimation hot path on one MI355X.

A step is one pdd_decimate call on device-resident synthetic input: voxel
grid, initial k-NN costs, removal rounds and finalisation, producing the kept
indices and the removal order.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, help="workload 1..5 (2: 20M-point scan, k=16, keep 10%%)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--round-frac", type=float, default=0.0)
    ap.add_argument("--voxel-log2", type=int, default=0)
    ap.add_argument("--b", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true", help="no per-50-round progress lines from the library")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2311_17604_amd import pdd, scangen

    t_gen = time.time()
    w = scangen.config(args.config, scale=args.scale)
    t_gen = time.time() - t_gen
    n = w.xyz.shape[0]
    x = torch.from_numpy(w.xyz).cuda()
    ctx = pdd.Context(0)
    kept = torch.empty(w.keep, dtype=torch.int32, device="cuda")
    order = torch.empty(n - w.keep, dtype=torch.int32, device="cuda")
    oc = torch.empty(n - w.keep, dtype=torch.int64, device="cuda")
    kw = dict(b=args.b, voxel_log2=args.voxel_log2, round_frac=args.round_frac, out=(kept, order, oc), timing=True,
              progress=not args.quiet)
    for i in range(args.warmup):
        pdd.decimate(ctx, x, w.keep, w.k, **kw)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phases = []
    for i in range(args.steps):
        pdd.decimate(ctx, x, w.keep, w.k, **kw)
        phases.append(ctx.timing())
        print("step %d done %s" % (i, phases[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    rec = {
        "metric": "input points decimated/s at 1 MI355X (learned+batched vs plain), bit-exact",
        "value": n * args.steps / dt,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "k": w.k, "keep": w.keep, "method": "plain",
                   "gen_s": round(t_gen, 2), "stats": st,
                   "phase_ms": {p: round(sum(ph[p] for ph in phases) / len(phases), 3) for p in phases[0]}},
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
