"""Throughput of the decimation hot path on one MI355X.

A step is one pdd_decimate call on device-resident synthetic input: voxel
grid, initial k-NN costs, removal rounds and finalisation, producing the kept
indices and the removal order (pdd_decimate_batch for the batch workload).
Before the timed steps the autotuner picks the list width, finest cell level
and round share by timed trials on a strided sample (not timed; reported in
config.autotune; the settings never change the result).  Prints one JSON
line with

  roofline      the k-NN cost phase (the LDS-tiled kernel knn_tile_k plus the
                shell search of its few uncertified points, knn_list_k):
                algorithmic bytes per launch (read one 16-byte point, write
                its K-entry list, cost and count) over the phase's duration
                from HIP events recorded on the library's stream; traffic
                from the rocprofv3 counter summary in profiles/ when it
                matches the workload, list width and kernel source;
  cpu_baseline  the CPU oracle (one core) on a bounded window of the same
                scan.
config.plain holds the same steps without the learned search region,
config.batched the batch workload at 1/16 size (256 scans): one autotuned
pdd_decimate_batch per step against the same scans one pdd_decimate at a
time, with the kept sets compared, and config.quality the measures of Sec. 6
on the kept points (pdd_quality_measure; not timed).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "knn_cost_counters.json")
KNN_SOURCES = ("paper_2311_17604_amd/csrc/knn.hip", "paper_2311_17604_amd/csrc/search.h")


def knn_source_hash() -> str:
    h = hashlib.sha256()
    for p in KNN_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per k-NN launch from the committed counter summary, or None
    when it is missing, for another workload or kernel instance, or for
    another kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("workload") != workload or c.get("kernel") != kernel or c.get("source_sha") != knn_source_hash():
        return None
    return c.get("traffic_bytes")


def cpu_baseline(w, rows_cols):
    """Oracle points/s on an angular window of the scan (rows x columns of the
    ray grid), one core."""
    import numpy as np

    from oracle import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    R, C = rows_cols
    r0, r1, c0, c1 = R * 2 // 5, R * 2 // 5 + R // 7, 0, C // 6
    idx = (np.arange(r0, r1)[:, None] * C + np.arange(c0, c1)[None, :]).ravel()
    P = np.ascontiguousarray(w.xyz[idx])
    keep = max(1, len(P) * w.keep // len(w.xyz))
    t = time.perf_counter()
    oracle.decimate(P, w.k, keep, b=8)
    dt = time.perf_counter() - t
    return {"value": len(P) / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": "rows %d-%d x columns %d-%d of the %dx%d ray grid (%d points, keep %d, k=%d), %.1f s"
                      % (r0, r1, c0, c1, R, C, len(P), keep, w.k, dt)}


GRIDS = {1: (500, 400), 2: (5000, 4000)}
BATCH_SCALE = 0.0625  # the batch workload beside the single-scan line: 256 scans, 1/16 sizes
QUALITY_R2 = [v * v for v in (100, 200, 300, 400, 500)]  # squared radii (mm^2) of the kept set's quality measures


def batch_compare(ctx, steps, warmup, learned):
    """The batch workload at 1/16 size (256 scans of 625 to 125k points):
    one autotuned pdd_decimate_batch per step (with the learned search region
    when `learned`) against the same scans decimated one pdd_decimate at a
    time (library defaults, plain), with the kept sets compared."""
    import numpy as np
    import torch

    from paper_2311_17604_amd import pdd, scangen
    w = scangen.config(4, scale=BATCH_SCALE)
    x = torch.from_numpy(w.xyz).cuda()
    n = len(w.xyz)
    tune = pdd.autotune_batch(ctx, x, w.offsets, w.keeps, w.k)
    kw = dict(b=tune["b"], voxel_log2=tune["voxel_log2"], round_frac=tune["round_frac"])
    for _ in range(warmup):
        pdd.decimate_batch(ctx, x, w.offsets, w.keeps, w.k, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        kb, _, _ = pdd.decimate_batch(ctx, x, w.offsets, w.keeps, w.k, **kw)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    if learned:
        pdd.pred_enable(ctx, False)
    parts = []
    t0 = time.perf_counter()
    for s in range(len(w.keeps)):
        a, b = int(w.offsets[s]), int(w.offsets[s + 1])
        k1, _, _ = pdd.decimate(ctx, x[a:b].contiguous(), int(w.keeps[s]), w.k)
        parts.append(k1)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    if learned:
        pdd.pred_enable(ctx, True, PRED_MARGIN)
    same = bool(np.array_equal(torch.cat(parts).cpu().numpy(), kb.cpu().numpy()))
    return {"workload": "%s@%g" % (w.name, BATCH_SCALE), "n": n, "clouds": int(len(w.keeps)),
            "value": n * steps / dtb, "ms_per_step": dtb * 1e3 / steps, "learned": learned, "autotune": tune,
            "one_by_one": {"value": n / dt1, "ms": dt1 * 1e3}, "same_kept": same}
PRED_MARGIN = 0.25


def train_predictor(ctx, k, b):
    """Trains the context's search-radius predictor for list width
    list(k + b) on scans of the 200k-scan generator (seeds 101-104, half the
    ray grid) and returns a summary."""
    import torch

    from paper_2311_17604_amd import pdd, scangen
    feats, tgts = [], []
    for seed in (101, 102, 103, 104):
        wt = scangen.config(1, scale=0.5, seed=seed)
        f, t = pdd.pred_samples(ctx, torch.from_numpy(wt.xyz).cuda(), k, b)
        feats.append(f)
        tgts.append(t)
    feat, tgt = torch.cat(feats), torch.cat(tgts)
    pdd.pred_set_weights(ctx, pdd.pred_init(11, float(tgt.mean().item())))
    losses = pdd.pred_train(ctx, feat, tgt, steps=1500, batch=128, lr=2e-3, tau=0.9, seed=5).cpu().numpy()
    return {"rows": int(feat.shape[0]), "loss_first": float(losses[:20].mean()),
            "loss_last": float(losses[-100:].mean()), "margin_log2": PRED_MARGIN}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, help="workload 1..5 (2: 20M-point scan, k=16, keep 10%%)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--round-frac", type=float, default=0.0)
    ap.add_argument("--voxel-log2", type=int, default=0)
    ap.add_argument("--b", type=int, default=0)
    ap.add_argument("--round-blocks", type=int, default=0, help="workgroups per round-kernel launch (0: library default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (by default b, voxel and round share are chosen first by timed trials "
                         "on a sample; not timed, reported as config.autotune)")
    ap.add_argument("--no-predictor", action="store_true",
                    help="skip the learned search-radius bound (by default it is trained first on k-NN radii of "
                         "scans from the 200k-scan generator, other seeds; not timed, reported as config.predictor)")
    ap.add_argument("--no-plain", action="store_true",
                    help="do not also time the plain configuration (no predictor) for comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="do not also time the batch workload (256 scans at 1/16 size, batched vs one at a time)")
    ap.add_argument("--quiet", action="store_true", help="no per-50-round progress lines from the library")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run four 1 GiB device-to-device copies (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs a decimation on one GPU and has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_17604_amd import pdd, scangen

    t_gen = time.time()
    w = scangen.config(args.config, scale=args.scale)
    t_gen = time.time() - t_gen
    n = w.xyz.shape[0]
    x = torch.from_numpy(w.xyz).cuda()
    ctx = pdd.Context(0)
    batch = w.offsets is not None
    tune = None
    if not args.no_autotune:
        t_tune = time.time()
        if batch:
            tune = pdd.autotune_batch(ctx, x, w.offsets, w.keeps, w.k, b=args.b, voxel_log2=args.voxel_log2,
                                      round_frac=args.round_frac)
        else:
            tune = pdd.autotune(ctx, x, w.keep, w.k, b=args.b, voxel_log2=args.voxel_log2,
                                round_frac=args.round_frac)
        tune["tune_s"] = round(time.time() - t_tune, 2)
        print("autotune: %s" % tune, file=sys.stderr, flush=True)
        args.b, args.voxel_log2, args.round_frac = tune["b"], tune["voxel_log2"], tune["round_frac"]
    pred = None
    if not args.no_predictor:
        t_tr = time.time()
        pred = train_predictor(ctx, w.k, args.b)
        pred["train_s"] = round(time.time() - t_tr, 2)
        print("predictor: %s" % pred, file=sys.stderr, flush=True)
    if batch:
        kw = dict(b=args.b, voxel_log2=args.voxel_log2, round_frac=args.round_frac, timing=True,
                  progress=not args.quiet, round_blocks=args.round_blocks)
        run = lambda: pdd.decimate_batch(ctx, x, w.offsets, w.keeps, w.k, **kw)  # noqa: E731
    else:
        kept = torch.empty(w.keep, dtype=torch.int32, device="cuda")
        order = torch.empty(n - w.keep, dtype=torch.int32, device="cuda")
        oc = torch.empty(n - w.keep, dtype=torch.int64, device="cuda")
        kw = dict(b=args.b, voxel_log2=args.voxel_log2, round_frac=args.round_frac, out=(kept, order, oc),
                  timing=True, progress=not args.quiet, round_blocks=args.round_blocks)
        run = lambda: pdd.decimate(ctx, x, w.keep, w.k, **kw)  # noqa: E731

    def timed(label):
        for i in range(args.warmup):
            run()
            print("%s warmup %d done" % (label, i), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phases = []
        for i in range(args.steps):
            run()
            phases.append(ctx.timing())
            print("%s step %d done %s" % (label, i, phases[-1]), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, phases

    plain = None
    if pred is not None and not args.no_plain:
        pdd.pred_enable(ctx, False)
        dtp, _ = timed("plain")
        plain = {"value": n * args.steps / dtp, "ms_per_step": dtp * 1e3 / args.steps}
    if pred is not None:
        pdd.pred_enable(ctx, True, PRED_MARGIN)
    dt, phases = timed("learned" if pred is not None else "plain")
    st = ctx.stats()
    ph = {p: round(sum(q[p] for q in phases) / len(phases), 3) for p in phases[0]}

    # k-NN cost kernel: one launch per step
    K = st["list_width"]
    bytes_per_point = 16 + 4 * K + 8 + 1
    algo = n * bytes_per_point
    knn_ms = ph["knn"]
    achieved = algo / (knn_ms * 1e-3) / 1e9
    workload = w.name if args.scale == 1.0 else "%s@%g" % (w.name, args.scale)
    kname = "knn_tile_k<%d,u32|u64>+knn_list_k<%d>" % (K, K)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, kname),
            "kernel": kname, "algorithmic_bytes_per_launch": algo,
            "bytes_per_point": bytes_per_point, "avg_launch_ms": knn_ms}

    quality = None
    if not batch:
        # the measures of Sec. 6 on the kept points of the last step (not
        # timed): density from the slope of neighbour count against area, R^2,
        # RMSE, and the smallest nearest-neighbour distance (Eq. 2)
        kidx = torch.sort(kept.long()).values
        kp = x[kidx].contiguous()
        tq = time.perf_counter()
        qs, _, _ = pdd.quality(ctx, kp, QUALITY_R2, with_counts=False)
        torch.cuda.synchronize()
        quality = {"points": int(kp.shape[0]), "radii_mm": [int(round(v ** 0.5)) for v in QUALITY_R2],
                   "mean_count": [round(v, 3) for v in qs["mean"]], "median_count": [f[3] for f in qs["fractiles"]],
                   "density_per_m2": round(qs["slope"], 2), "r_squared": round(qs["r_squared"], 4),
                   "rmse": round(qs["rmse"], 3), "nn_min_mm": round(qs["nn2_min"] ** 0.5, 2),
                   "ms": round((time.perf_counter() - tq) * 1e3, 1)}

    batched = None
    if not args.no_batch and not batch:
        print("batch workload: batched vs one at a time", file=sys.stderr, flush=True)
        batched = batch_compare(ctx, args.steps, args.warmup, pred is not None)

    cpu = None
    if not args.no_cpu_baseline and args.config in GRIDS and args.scale == 1.0:
        print("cpu baseline: oracle on a window of the scan", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, GRIDS[args.config])

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
        "config": {"workload": workload, "n": n, "k": w.k, "keep": w.keep,
                   "method": "+".join([m for m, on in (("batched", batch), ("autotuned", tune is not None),
                                                        ("learned", pred is not None)) if on]) or "plain",
                   "clouds": int(len(w.keeps)) if batch else 1, "autotune": tune, "predictor": pred,
                   "plain": plain, "batched": batched, "quality": quality,
                   "gen_s": round(t_gen, 2), "stats": st, "phase_ms": ph},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
