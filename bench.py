"""Benchmark of the MAM hot path on one MI355X.

One step = one deterministic MAM iteration (Alg. 1: every measure, every
column) over the whole problem, inputs resident in HBM.  The workload is the
balanced sparse barycenter problem: R = 64 x 64 = 4096 barycenter support
points, M = 32 image-like measures whose supports are the pixels with blob
density above 1e-3 (S^m uneven, T ~ 9.8e4 columns), squared Euclidean grid
cost gathered by pixel index, rho = 1, plans in FP32 (thresholds, marginals
and barycenter in FP64).  The default run times the 500 iterations that
problem is quoted at, then the same 500 iterations with FP64 plans, and
reports the FP32-vs-FP64 barycenter difference.

Prints one JSON line:  metric, value (plan-entry updates per second), the
roofline of the dominant kernel (the column kernel, timed with HIP events on
the launch stream), the FP64 run and the oracle's CPU rate on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps 500] [--warmup 10] [--no-cpu] [--copy-probe]
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

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_column_kernel_balanced_sparse_K64_M32.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2309_05315_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(p) -> int:
    """Bytes one column-kernel launch must move at minimum: every plan entry
    read and written once, every distinct cost entry read once, q read once."""
    eb = 4 if p.dtype == "f32" else 8
    return eb * (2 * p.R * p.T + p.R * p.distinct_cost_columns() + p.T)


def run_gpu(p, steps, warmup, torch, mam):
    s = mam.solver_for(p, device="cuda:0")
    s.init()
    s.iterate(warmup)
    torch.cuda.synchronize()
    # timed region: exactly `steps` iterations, synchronised on both sides
    t0 = time.perf_counter()
    s.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pbar = s.barycenter().cpu().numpy()
    # dominant-kernel duration: HIP events around every column-kernel launch
    s.timing(True)
    s.iterate(min(steps, 100))
    col_ms, n = s.timing_read()
    s.timing(False)
    sched = s.schedule()
    s.close()
    del s
    torch.cuda.empty_cache()
    return dt, pbar, col_ms / max(n, 1), n, sched


def cpu_baseline(p, n_measures):
    import numpy as np
    from oracle import mam_oracle as O
    k = min(n_measures, p.M)
    cost = [p.cost_block(m) for m in range(k)]
    q = [p.q_block(m) for m in range(k)]
    t0 = time.perf_counter()
    O.mam(cost, q, p.rho, p.gamma, 1)
    dt = time.perf_counter() - t0
    entries = p.R * sum(p.S[:k])
    return {"value": entries / dt, "unit": "plan-entry updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 iteration of the FP64 numpy oracle over the first {k} of {p.M} measures "
                      f"({entries:.3e} plan entries, {dt:.1f} s, single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--cpu-measures", type=int, default=12)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2309_05315_amd import inputs, mam

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    mam.lib()

    p32 = inputs.balanced_sparse(dtype="f32")
    log(f"workload {p32.name}: R={p32.R} M={p32.M} T={p32.T} S in [{min(p32.S)}, {max(p32.S)}]")
    dt32, pb32, col_ms32, ncol, sched = run_gpu(p32, args.steps, args.warmup, torch, mam)
    entries = p32.R * p32.T
    value = entries * args.steps / dt32
    ab = algorithmic_bytes(p32)
    achieved = ab / (col_ms32 * 1e-3) / 1e9
    log(f"fp32: {dt32 / args.steps * 1e3:.4f} ms/iter, column kernel {col_ms32:.4f} ms, "
        f"{achieved:.0f} GB/s algorithmic, schedule {sched}")

    fp64 = None
    if not args.no_fp64:
        p64 = inputs.balanced_sparse(dtype="f64")
        dt64, pb64, col_ms64, _, sched64 = run_gpu(p64, args.steps, args.warmup, torch, mam)
        ab64 = algorithmic_bytes(p64)
        fp64 = {
            "value": entries * args.steps / dt64,
            "ms_per_step": dt64 / args.steps * 1e3,
            "column_kernel_ms": col_ms64,
            "achieved_GBs": ab64 / (col_ms64 * 1e-3) / 1e9,
            "fp32_speedup": dt64 / dt32,
            "barycenter_rel_l1_fp32_vs_fp64": float(np.abs(pb32 - pb64).sum() / np.abs(pb64).sum()),
            "barycenter_rel_max_fp32_vs_fp64": float(np.abs(pb32 - pb64).max() / np.abs(pb64).max()),
        }
        log(f"fp64: {fp64['ms_per_step']:.4f} ms/iter; fp32/fp64 barycenter rel L1 "
            f"{fp64['barycenter_rel_l1_fp32_vs_fp64']:.3e}")

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")

    if args.copy_probe:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {4 * n} bytes copied")

    cpu = None if args.no_cpu else cpu_baseline(p32, args.cpu_measures)

    out = {
        "metric": "plan-entry updates/s (FP32 plans, FP64 thresholds) + HBM GB/s fraction of the column kernel",
        "value": value,
        "unit": "plan-entry updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "balanced sparse WB, 64x64 grid (R=4096), M=32 thresholded blob "
                               "measures, indexed squared-Euclidean grid cost, rho=1, FP32 plans",
                   "R": p32.R, "M": p32.M, "T": p32.T, "S_min": min(p32.S), "S_max": max(p32.S),
                   "iterations": args.steps, "schedule": sched},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "column_kernel", "algorithmic_bytes_per_launch": ab,
                     "avg_launch_ms": col_ms32, "launches_timed": ncol},
        "fp64": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
