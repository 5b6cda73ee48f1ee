"""Write the full-iteration-count oracle references under tests/golden/fullk/.

    python tests/golden/make_fullk_refs.py [--workers 8] [name ...]

Each reference is the FP64 CPU oracle (Alg. 1, ``oracle.mam_parallel``: the
paper's scheme of one process per group of measures, equal bit for bit to
the one-process oracle) run on a seeded synthetic workload for the number of
iterations that workload is stated at.  Nothing here runs or reads the HIP
path: inputs come from ``paper_2309_05315_amd.inputs`` (generators only) and
every stored number from ``oracle``.

Per reference, ``<name>.npz`` holds p_bar (R) and pm (M x R, the marginals
p^(m) of theta^K), and ``index.json`` holds the iteration count, a hash of
the inputs (so a test can tell when a generator changed), the last damping
t^k and the figures of the last iteration: W_hat = sum_m <c^(m), pi_hat^(m)>,
dist_L(pi_hat), the measure residual max_s |sum_r pi_hat_rs - q_s| and
||theta^K - theta^(K-1)||_inf.
"""
from __future__ import annotations

import argparse
import functools
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.mam_parallel import mam_parallel  # noqa: E402
from paper_2309_05315_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "fullk")
INDEX = os.path.join(OUT, "index.json")


def adjoint_forward(**kw):
    """The reverse-mode workload's forward problem (its target is not needed)."""
    return inputs.adjoint_problem(**kw)[0]


def batch_member(index: int, **kw):
    """Problem ``index`` of the 256-problem batch."""
    return inputs.batched_problems(**kw)[index]


def batch_sample():
    """One problem from each band of sizes of the batch (R <= 121, 144-256,
    289-484, 529-784, 841-1024) and the batch's largest problem (most plan
    entries): the first problem of each band in batch order."""
    ps = inputs.batched_problems()
    bands = [(0, 121), (144, 256), (289, 484), (529, 784), (841, 1024)]
    pick = []
    for lo, hi in bands:
        pick.append(next(i for i, p in enumerate(ps) if lo <= p.R <= hi))
    big = max(range(len(ps)), key=lambda i: ps[i].R * ps[i].T)
    if big not in pick:
        pick.append(big)
    return pick


def workloads():
    """name -> (builder, iterations, what it stands for)."""
    w = {
        "balanced_sparse_K64_M32_f32_k500": (
            functools.partial(inputs.balanced_sparse, dtype="f32"), 500,
            "balanced sparse 64x64 grid, 32 measures, FP32 inputs, 500 iterations"),
        "balanced_sparse_K64_M32_f64_k500": (
            functools.partial(inputs.balanced_sparse, dtype="f64"), 500,
            "balanced sparse 64x64 grid, 32 measures, FP64 inputs, 500 iterations"),
        "balanced_sparse_K32_M8_f32_k500": (
            functools.partial(inputs.balanced_sparse, K=32, M=8, dtype="f32"), 500,
            "the same at quarter scale (32x32 grid, 8 measures), FP32 inputs"),
        "balanced_sparse_K32_M8_f64_k500": (
            functools.partial(inputs.balanced_sparse, K=32, M=8, dtype="f64"), 500,
            "the same at quarter scale, FP64 inputs"),
        "unbalanced_dense_K32_M50_f32_k1000": (
            functools.partial(inputs.unbalanced_dense, dtype="f32"), 1000,
            "unbalanced 32x32 grid, 50 measures, gamma = 0.01, FP32 inputs, 1000 iterations"),
        "unbalanced_dense_K16_M12_f32_k1000": (
            functools.partial(inputs.unbalanced_dense, K=16, M=12, dtype="f32"), 1000,
            "the same at quarter scale (16x16 grid, 12 measures)"),
        "adjoint_K64_M8_f32_k100": (
            functools.partial(adjoint_forward, dtype="f32"), 100,
            "the reverse-mode workload's forward: 64x64 grid, 8 dense measures, FP32 inputs, 100 iterations"),
    }
    for i in batch_sample():
        w[f"batch256_p{i}_f32_k300"] = (
            functools.partial(batch_member, i), 300,
            f"problem {i} of the 256-problem batch, FP32 inputs, 300 iterations")
    return w


def inputs_hash(p) -> str:
    """sha256 of everything the iteration reads: sizes, rho, gamma, weights,
    cost and the cost index."""
    h = hashlib.sha256()
    h.update(json.dumps({"R": p.R, "S": list(map(int, p.S)), "rho": p.rho, "gamma": p.gamma,
                         "dtype": p.dtype}).encode())
    h.update(np.ascontiguousarray(p.q, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(p.cost, dtype=np.float64).tobytes())
    if p.col_index is not None:
        h.update(np.ascontiguousarray(p.col_index, dtype=np.int32).tobytes())
    return h.hexdigest()


def load_index() -> dict:
    if os.path.exists(INDEX):
        with open(INDEX) as f:
            return json.load(f)
    return {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 4)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    todo = workloads()
    names = args.names or list(todo)
    os.makedirs(OUT, exist_ok=True)
    for name in names:
        build, iters, what = todo[name]
        p = build()
        print(f"{name}: R={p.R} M={p.M} T={p.T} iters={iters} ({what})", flush=True)
        t0 = time.perf_counter()
        ref = mam_parallel(build, iters, args.workers, log=lambda s: print(s, flush=True))
        dt = time.perf_counter() - t0
        np.savez_compressed(os.path.join(OUT, name + ".npz"), p_bar=ref["p_bar"], pm=ref["pm"])
        idx = load_index()
        idx[name] = {
            "what": what, "iters": iters, "R": p.R, "M": p.M, "T": p.T, "dtype": p.dtype,
            "rho": p.rho, "gamma": p.gamma, "inputs_sha256": inputs_hash(p),
            "t_last": ref["t"], "W_hat": ref["W_hat"], "dist_L": ref["dist_L"],
            "meas_resid": ref["meas_resid"], "dtheta_inf": ref["dtheta_inf"],
            "oracle_seconds": round(dt, 1), "workers": min(args.workers, p.M),
        }
        with open(INDEX, "w") as f:
            json.dump(idx, f, indent=1, sort_keys=True)
            f.write("\n")
        print(f"  done in {dt:.0f} s: W_hat={ref['W_hat']:.10g} dist_L={ref['dist_L']:.4g}", flush=True)


if __name__ == "__main__":
    main()
