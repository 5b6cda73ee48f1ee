"""Benchmark of the MAM hot path on one MI355X.

One step = one deterministic MAM iteration (Alg. 1: every measure, every
column) over the whole problem, inputs resident in HBM.  The workload is the
balanced sparse barycenter problem: R = 64 x 64 = 4096 barycenter support
points, M = 32 image-like measures whose supports are the pixels with blob
density above 1e-3 (S^m uneven, T ~ 9.8e4 columns), squared Euclidean grid
cost gathered by pixel index, rho = 1, plans in FP32 (thresholds, marginals
and barycenter in FP64).  The default run times the 500 iterations that
problem is quoted at, then the same 500 iterations with FP64 plans, and
reports the FP32-vs-FP64 barycenter difference.  Shorter runs of the other
workloads (balanced FP64 with graph replay, unbalanced, unbalanced with the
measure constraints relaxed, a batch of 256 problems, the randomized variant, on-device stopping tests, the free-support
workload on the long-column path, the reverse mode) are reported under
"extras".

Prints one JSON line:  metric, value (plan-entry updates per second), the
roofline of the dominant kernel (the column kernel, timed with HIP events on
the launch stream), the FP64 run and the oracle's CPU rate on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps 500] [--warmup 10] [--no-cpu]
                    [--no-extras | --extras free_support,adjoint,...]
"""
from __future__ import annotations

import argparse
import dataclasses
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
    """Hash of the column kernel's device sources (its template, instances and
    dispatch); the launch schedule is compared separately."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2309_05315_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name in ("mam_kernels.hpp", "mam_instances.hpp", "mam_dispatch.hpp") or \
                (name.startswith(("col_f32", "col_f64")) and name.endswith(".hip")):
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


def final_state(p, iters, torch, mam, relaxed=False):
    """The state the timed run reached, recomputed untimed with diagnostics
    on its last iteration: objective W_hat = sum c pi_hat, dist_L (the
    marginals' distance to agreement), the measure-constraint residual, the
    threshold passes and active entries per column."""
    s = mam.solver_for(p, device="cuda:0", diag=True, relaxed=relaxed)
    s.init()
    s.iterate(iters)
    d = s.diagnostics()
    s.close()
    del s
    torch.cuda.empty_cache()
    return {k: d[k] for k in ("iterations", "W_hat", "dist_L", "meas_resid", "dtheta_inf",
                              "rounds_per_column", "active_per_column")}


def copy_ceiling(torch, mam, nbytes=1 << 30):
    """The device's read-plus-write streaming ceiling: the library's copy
    probe (non-temporal 16-byte loads and stores, grid-stride) over two
    1 GiB buffers at several workgroup counts, timed with HIP events on the
    launch stream; the best is the ceiling."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    res = {}
    for nwg in (1024, 4096, 16384, 32768):
        for _ in range(2):
            mam.stream_copy(b, a, nwg)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            mam.stream_copy(b, a, nwg)
        e1.record()
        torch.cuda.synchronize()
        res[nwg] = 2 * nbytes / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    best = max(res, key=res.get)
    return {"GBs": res[best], "workgroups": best, "by_workgroups": {str(k): v for k, v in res.items()},
            "bytes_each_way": nbytes}


FULLK = os.path.join(ROOT, "tests", "golden", "fullk")


def error_vs_oracle(p, torch, mam):
    """The FP32 plans' error against the FP64 oracle at the workload's
    stated 500 iterations: the oracle's barycenter, marginals and last-
    iteration figures are stored references (written by
    tests/golden/make_fullk_refs.py, which runs only the oracle); the device
    runs the same 500 iterations from the same start, untimed, with
    diagnostics on the last."""
    import numpy as np
    name = "balanced_sparse_K64_M32_f32_k500"
    try:
        with open(os.path.join(FULLK, "index.json")) as f:
            meta = json.load(f)[name]
        ref = np.load(os.path.join(FULLK, name + ".npz"))
    except (OSError, KeyError) as e:
        return {"error": f"reference {name} not available: {e}"}
    K = int(meta["iters"])
    s = mam.solver_for(p, device="cuda:0", diag=True)
    s.init()
    s.iterate(K)
    d = s.diagnostics()
    pb = s.barycenter().cpu().numpy()
    pm = s.marginals().cpu().numpy()
    s.close()
    del s
    torch.cuda.empty_cache()
    po, pmo = ref["p_bar"], ref["pm"]
    return {
        "iterations": K,
        "barycenter_rel_l1": float(np.abs(pb - po).sum() / np.abs(po).sum()),
        "barycenter_rel_max": float(np.abs(pb - po).max() / np.abs(po).max()),
        "marginals_rel_max": float(np.abs(pm - pmo).max() / np.abs(pmo).max()),
        "objective_rel": abs(d["W_hat"] - meta["W_hat"]) / abs(meta["W_hat"]),
        "marginal_residual_dist_L": {"device": d["dist_L"], "oracle": meta["dist_L"],
                                     "rel": abs(d["dist_L"] - meta["dist_L"]) / abs(meta["dist_L"])},
        "measure_residual": {"device": d["meas_resid"], "oracle": meta["meas_resid"]},
        "reference": f"tests/golden/fullk/{name}.npz",
    }


def host_cpu() -> str:
    """The host's CPU model and logical core count, for the baseline records."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores"


def cpu_baseline(p, n_measures, iters=2):
    from oracle import mam_oracle as O
    k = min(n_measures, p.M)
    cost = [p.cost_block(m) for m in range(k)]
    q = [p.q_block(m) for m in range(k)]
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one core, BLAS included
        t0 = time.perf_counter()
        O.mam(cost, q, p.rho, p.gamma, iters)
        dt = time.perf_counter() - t0
    entries = p.R * sum(p.S[:k]) * iters
    return {"value": entries / dt, "unit": "plan-entry updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iteration(s) of the FP64 numpy oracle over the first {k} of {p.M} measures "
                      f"({entries:.3e} plan-entry updates, {dt:.1f} s, single thread on {host_cpu()})"}


def _oracle_measures_worker(args):
    """One process of the paper's parallel scheme: Step 2 and the marginal of
    Step 3 for its measures, from theta^0 = q_s/R (the problem is rebuilt
    here, so nothing large crosses the process boundary).  Returns the
    seconds of its numpy work and its plan entries."""
    ms, dtype = args
    import numpy as np
    from oracle import mam_oracle as O
    from paper_2309_05315_amd import inputs
    p = inputs.balanced_sparse(dtype=dtype)
    a = O.averaging_weights(p.S)
    pm = np.stack([np.full(p.R, float(p.q_block(m).sum()) / p.R) for m in range(p.M)])
    pbar = (a[:, None] * pm).sum(axis=0)
    t, _ = O.damping(pbar, pm, p.S, p.rho, p.gamma)
    blocks = {m: p.cost_block(m) for m in ms}
    t0 = time.perf_counter()
    for m in ms:
        q = p.q_block(m)
        theta = np.repeat((q / p.R)[None, :], p.R, axis=0)
        corr = t * (pbar - pm[m]) / p.S[m]
        w = theta + 2.0 * corr[:, None] - blocks[m] / p.rho
        ph = O.proj_simplex_sort(w, q)[0]
        (ph - corr[:, None]).sum(axis=1)
    return time.perf_counter() - t0, p.R * sum(p.S[m] for m in ms)


def cpu_baseline_parallel(p, workers):
    """The paper's own parallel scheme (one process per group of measures,
    Step 2 in parallel, the averaging as the gathering step): one iteration
    over all measures on 'workers' host processes; the wall time is the
    slowest process's."""
    import multiprocessing as mp
    parts = [list(range(w, p.M, workers)) for w in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_measures_worker, [(ms, p.dtype) for ms in parts])
    wall = max(dt for dt, _ in res)
    entries = sum(e for _, e in res)
    return {"value": entries / wall, "unit": "plan-entry updates/s", "cores": workers, "kind": "oracle",
            "sample": f"1 iteration of the FP64 numpy oracle over all {p.M} measures, {workers} processes "
                      f"(measures dealt round robin; wall time = the slowest process, {wall:.2f} s) "
                      f"on {host_cpu()}"}


EXTRAS = ("balanced_plain", "unbalanced", "relaxed", "batch", "randomized", "stopping", "free_support",
          "adjoint", "large_rho")


def extra_workloads(torch, mam, inputs, log, only=None):
    """The other workloads of the hot path, timed briefly (informational);
    ``only``: the names (of EXTRAS) to run, all by default."""
    import numpy as np
    out = {}
    sync = torch.cuda.synchronize

    def timed(fn):
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        return time.perf_counter() - t0

    def want(name):
        return only is None or name in only

    p1 = inputs.balanced_plain()
    p2 = inputs.balanced_sparse(dtype="f32")

    if want("balanced_plain"):
        # balanced, FP64, 16x16 grid, 4 measures: launch-bound; eager vs graph replay
        s = mam.solver_for(p1)
        s.init()
        s.iterate(10)
        eager = timed(lambda: s.iterate(p1.iters)) / p1.iters
        s.graph(50)
        s.init()
        s.iterate(50)
        graph = timed(lambda: s.iterate(p1.iters)) / p1.iters
        s.close()
        out["balanced_plain_K16_M4_f64"] = {"iterations": p1.iters, "ms_per_iter_eager": eager * 1e3,
                                            "ms_per_iter_graph": graph * 1e3}
        log(f"balanced plain: {eager * 1e3:.4f} ms/iter eager, {graph * 1e3:.4f} ms/iter graph")

    if want("unbalanced"):
        # unbalanced, FP32, 32x32 grid, 50 measures, gamma = 0.01
        p3 = inputs.unbalanced_dense()
        s = mam.solver_for(p3)
        s.init()
        s.iterate(10)
        dt = timed(lambda: s.iterate(p3.iters)) / p3.iters
        s.timing(True)
        s.iterate(100)
        col, n = s.timing_read()
        s.timing(False)
        # the same iterations replayed from a captured graph (50 per launch)
        s.graph(50)
        s.init()
        s.iterate(50)
        dtg = timed(lambda: s.iterate(p3.iters)) / p3.iters
        s.close()
        # the damping t^k of every iteration of a run from the start (Alg. 1,
        # eq. (Unbalanced-prox)): how often the unbalanced rule damps
        s = mam.solver_for(p3, diag=True)
        s.init()
        ts = []
        for _ in range(p3.iters):
            s.iterate(1)
            ts.append(s.diagnostics()["t"])
        s.close()
        ts = np.asarray(ts)
        ab = algorithmic_bytes(p3)
        out["unbalanced_K32_M50_f32"] = {"iterations": p3.iters, "ms_per_iter": dt * 1e3,
                                         "ms_per_iter_graph": dtg * 1e3,
                                         "column_kernel_ms": col / n,
                                         "column_kernel_GBs": ab / (col / n * 1e-3) / 1e9,
                                         "damped_fraction": float(np.mean(ts < 1.0)),
                                         "t_min": float(ts.min()), "t_last": float(ts[-1]),
                                         "first_undamped_iteration": int(np.argmax(ts >= 1.0)) + 1 if np.any(ts >= 1.0) else None}
        log(f"unbalanced: {dt * 1e3:.4f} ms/iter, {dtg * 1e3:.4f} ms/iter graph, column kernel {col / n:.4f} ms, "
            f"t < 1 in {np.mean(ts < 1.0):.1%} of {p3.iters} iterations")

    if want("relaxed"):
        # the full unbalanced extension: measure constraints relaxed to
        # sum_r pi_rs <= q_s, the penalty of unassigned mass entering as the
        # shifted cost c - eta.  Random supports (so no measure point sits on
        # a barycenter point and leaving mass unassigned can be the cheaper
        # choice): R = 1024 barycenter points, 32 measures of 1024 points
        # with masses in [0.5, 1.5], one shared cost, gamma = 0.2, FP32
        eta, gam, n_it = 0.002, 0.2, 300
        rng = np.random.default_rng(55)
        masses = list(rng.uniform(0.5, 1.5, size=32))
        p5 = inputs.tiny_problem(55, R=1024, S=[1024] * 32, dtype="f32", masses=masses, gamma=gam, shared=True)
        p5 = dataclasses.replace(p5, cost=(p5.cost - eta).astype(np.float32).astype(np.float64))
        s = mam.solver_for(p5, relaxed=True)
        s.init()
        s.iterate(10)
        dt = timed(lambda: s.iterate(n_it)) / n_it
        s.timing(True)
        s.iterate(100)
        col, n = s.timing_read()
        s.timing(False)
        s.init()
        s.iterate(n_it)
        pb = s.barycenter().cpu().numpy()
        s.close()
        # the same iterations with the measure constraints kept: how much the
        # relaxation changes the barycenter
        s = mam.solver_for(p5)
        s.init()
        s.iterate(n_it)
        pb0 = s.barycenter().cpu().numpy()
        s.close()
        d = final_state(p5, n_it, torch, mam, relaxed=True)
        out["relaxed_R1024_M32_f32"] = {
            "eta": eta, "gamma": gam, "iterations": n_it, "ms_per_iter": dt * 1e3,
            "plan_entry_updates_per_s": p5.R * p5.T / dt, "column_kernel_ms": col / n,
            "column_kernel_GBs": algorithmic_bytes(p5) / (col / n * 1e-3) / 1e9,
            "barycenter_mass": float(pb.sum()), "barycenter_mass_constraints_kept": float(pb0.sum()),
            "barycenter_rel_diff_to_constraints_kept": float(np.abs(pb - pb0).max() / np.abs(pb0).max()),
            "state": d}
        log(f"relaxed (eta = {eta}): {dt * 1e3:.4f} ms/iter, column kernel {col / n:.4f} ms; barycenter mass "
            f"{pb.sum():.4f} against {pb0.sum():.4f} with the constraints kept; excess over q {d['meas_resid']:.2e}")

    if want("batch"):
        # 256 independent problems (R = k^2, k in 8..32, M in 2..8), FP32, autotuned
        # schedules per shape group, graph replay
        from paper_2309_05315_amd import autotune
        probs = inputs.batched_problems()
        t0 = time.perf_counter()
        scheds = autotune.tune_batch(probs)
        tune_s = time.perf_counter() - t0
        b = mam.Batch(probs, schedules=scheds)
        b.graph(25)
        b.init()
        b.iterate(25)
        iters4 = probs[0].iters
        dt = timed(lambda: b.iterate(iters4)) / iters4
        b.graph(0)
        b.timing(True)
        b.iterate(50)
        col, n = b.timing_read()
        b.close()
        ab = sum(algorithmic_bytes(p) for p in probs)
        out["batch_256_f32"] = {"problems": len(probs), "iterations": iters4, "ms_per_iter_graph": dt * 1e3,
                                "autotune_s": tune_s, "schedules": {str(g): v for g, v in scheds.items()},
                                "column_kernels_ms": col / n, "column_kernels_GBs": ab / (col / n * 1e-3) / 1e9,
                                "plan_entries": int(sum(p.R * p.T for p in probs))}
        log(f"batch of {len(probs)}: {dt * 1e3:.4f} ms/iter (graph), column kernels {col / n:.4f} ms")

    if want("randomized"):
        # randomized variant on the benchmark workload: 4 bundles of 8 measures,
        # drawn with probability proportional to alpha_m = 1/M (the same seeded draws
        # for every run)
        bundles = [list(range(i, p2.M, 4)) for i in range(4)]
        bundle_of = [m % 4 for m in range(p2.M)]
        seq = inputs.bundle_sequence(bundles, 200, seed=0)
        s = mam.solver_for(p2)
        s.init()
        s.set_bundles(bundle_of)
        s.iterate_bundles(seq[:20])
        dt = timed(lambda: s.iterate_bundles(seq[20:]))
        n_it = len(seq) - 20
        ent = sum(p2.R * sum(p2.S[m] for m in bundles[b]) for b in seq[20:])
        s.close()
        out["randomized_4_bundles_K64_M32_f32"] = {
            "iterations": n_it, "ms_per_iter": dt / n_it * 1e3, "plan_entry_updates_per_s": ent / dt,
            "entries_per_iter": ent / n_it}
        log(f"randomized, 4 bundles: {dt / n_it * 1e3:.4f} ms/iter, {ent / dt:.3e} entries/s")

    if want("stopping"):
        # stopping tests on the device (Sec. 5): the cost of a check every 10
        # iterations against plain iterations (graph replay in both), on the
        # benchmark workload and on the launch-bound 16x16 problem, and the time a
        # run of at most 20000 iterations takes when its first check stops it
        res = {}
        for name, prob in (("K64_M32_f32", p2), ("K16_M4_f64", p1)):
            s = mam.solver_for(prob)
            s.graph(10)
            s.init()
            s.iterate(20)
            r_ = {"plain_ms_per_iter": timed(lambda: s.iterate(200)) / 200 * 1e3}
            for test in ("dp", "dist", "dtheta"):
                s.init()
                s.iterate_until(20, test, -1.0, 10)
                r_[f"{test}_every_10_ms_per_iter"] = timed(lambda: s.iterate_until(200, test, -1.0, 10)) / 200 * 1e3
            s.init()
            got = {}
            r_["stop_at_first_check_ms"] = timed(lambda: got.update(s.iterate_until(20000, "dp", float("inf"), 10))) * 1e3
            r_["stop_at_first_check_iterations"] = got["iterations"]
            s.close()
            res[name] = r_
            log(f"stopping tests {name}: plain {r_['plain_ms_per_iter']:.4f} ms/iter, with checks every 10: "
                f"dp {r_['dp_every_10_ms_per_iter']:.4f}, dist {r_['dist_every_10_ms_per_iter']:.4f}, "
                f"dtheta {r_['dtheta_every_10_ms_per_iter']:.4f}; stop at the first check of 20000: "
                f"{r_['stop_at_first_check_ms']:.2f} ms")
        out["stopping_tests"] = res

    if want("free_support"):
        # free-support barycenter (Theorem c): 10 nested-ellipse 60x60 images,
        # R = 349,281 support points, T = 36,000 columns, FP32 plans (50 GB):
        # the long-column path (row tiles, candidate slots, per-column thresholds)
        pf = inputs.free_support(dtype="f32")
        res = {"R": pf.R, "M": pf.M, "T": pf.T, "plans_GB": pf.T * pf.R * 4 / 1e9}
        for mode, grid, sparse in (("stored_cost", False, False), ("grid_cost", True, False),
                                   ("stored_cost_sparse_store", False, True), ("grid_cost_sparse_store", True, True)):
            # sparse store: between the iterations of a call the plans are
            # -b plus the entries above lambda; the timed call ends with the
            # write-back of all 50 GB
            s = mam.solver_for(pf, grid=grid, sparse_store=sparse)
            sc = s.schedule()
            s.init()
            s.iterate(3)
            n_it = 20
            dt = timed(lambda: s.iterate(n_it)) / n_it
            s.timing(True)
            s.iterate(5)
            col, n = s.timing_read()
            s.timing(False)
            sup = {}
            if grid and not sparse:
                # the support step (Prop. 4): one more iteration, then the
                # alpha-weighted means of the pixel centres under its plans
                zt = torch.from_numpy(np.tile(pf.zeta, (pf.M, 1))).cuda()
                xt = torch.from_numpy(pf.xi.copy()).cuda()
                al = [1.0 / pf.M] * pf.M
                s.support_update(al, zt, xt)
                t_sup = min(timed(lambda: s.support_update(al, zt, xt)) for _ in range(3))
                sup = {"support_step_ms": t_sup * 1e3, "support_passes_ms": (t_sup - dt) * 1e3,
                       "support_workspace_GB": s.support_workspace.numel() / 1e9}
                log(f"free support: support step {t_sup * 1e3:.2f} ms with its iteration, "
                    f"{(t_sup - dt) * 1e3:.2f} ms for the two passes")
            ws = s.workspace.numel()
            s.close()
            del s
            torch.cuda.empty_cache()
            # algorithmic bytes of a dense iteration: theta read and written, the
            # distinct cost read once (none when the kernels form it from the
            # grid), q; the sparse store does not move theta, so no rate is
            # given for it (its column kernels time excludes the write-back,
            # its ms_per_iter includes it)
            abf = 4 * (2 * pf.R * pf.T + (0 if grid else pf.R * pf.distinct_cost_columns()) + pf.T)
            gbs = None if sparse else abf / (col / n * 1e-3) / 1e9
            res[mode] = {"iterations": n_it, "ms_per_iter": dt * 1e3, "plan_entry_updates_per_s": pf.R * pf.T / dt,
                         "column_kernels_ms": col / n, "algorithmic_bytes_per_iter": abf,
                         "column_kernels_GBs": gbs, "workspace_GB": ws / 1e9,
                         "rows_per_tile": sc["rows_per_tile"], "candidate_slots": sc["candidate_slots"],
                         "workgroups": sc["workgroups"], **sup}
            log(f"free support R={pf.R} T={pf.T} ({mode}): {dt * 1e3:.2f} ms/iter, {pf.R * pf.T / dt:.3e} entries/s, "
                f"column kernels {col / n:.2f} ms" + (f" ({gbs:.0f} GB/s algorithmic)" if gbs else ""))
        # the figures the free-support experiment reports (Sec. 6.3): the plan
        # objective W_hat and dist_L(pi_hat) of the last iteration, from the
        # long-column path's own diagnostics (outside every timed region)
        s = mam.solver_for(pf, grid=True, sparse_store=True, diag=True)
        s.init()
        n_d = 50
        s.iterate(n_d)
        d = s.diagnostics()
        s.close()
        del s
        torch.cuda.empty_cache()
        res["state_after_50"] = {k: (None if isinstance(v, float) and v != v else v) for k, v in d.items()}
        log(f"free support after {n_d} iterations: W_hat {d['W_hat']:.6e}, dist_L {d['dist_L']:.3e}, "
            f"measure residual {d['meas_resid']:.1e}")
        out["free_support_K60_M10_f32"] = res

    if want("adjoint"):
        # reverse mode: 64x64 grid, 8 measures, 100 iterations, FP32, loss ||p_bar - target||^2
        p5, tgt = inputs.adjoint_problem()
        tg = torch.as_tensor(tgt, device="cuda:0")
        res = {"iterations": p5.iters}
        for ck in (10, 0):
            s = mam.solver_for(p5)
            s.init()
            rec = timed(lambda: s.record(p5.iters, ck))
            g = 2.0 * (s.barycenter() - tg)
            s.backward(g)
            s.timing(True)
            bwd = timed(lambda: s.backward(g))
            ak, n = s.timing_read()
            sc = s.schedule()
            ws = s.adj_workspace.numel()
            s.close()
            res[f"ckpt_every_{ck}"] = {"record_ms": rec * 1e3, "backward_ms": bwd * 1e3,
                                       "adjoint_kernel_us": ak / n * 1e3, "adjoint_workspace_GB": ws / 1e9}
            log(f"adjoint ckpt_every={ck}: record {rec * 1e3:.1f} ms, backward {bwd * 1e3:.1f} ms, "
                f"adjoint kernel {ak / n * 1e3:.1f} us")
        # algorithmic bytes of one reverse column step: the active-set masks of
        # two iterations, q's adjoint (read and write), and for every active
        # entry the sparse adjoint (read, write) and the cost adjoint (read, write)
        s = mam.solver_for(p5, diag=True)
        s.init()
        s.iterate(p5.iters)
        act = s.diagnostics()["active_per_column"]
        s.close()
        mld = sc["threads_per_column"] * (1 if sc["values_per_thread"] <= 8 else 2)
        abytes = 2 * p5.T * mld + 16 * p5.T + 32 * act * p5.T
        us = res["ckpt_every_0"]["adjoint_kernel_us"]
        res["adjoint_kernel_roofline"] = {"bound": "hbm", "algorithmic_bytes_per_launch": abytes,
                                          "active_entries_per_column": act,
                                          "achieved": abytes / (us * 1e-6) / 1e9, "peak": PEAK_HBM_GBS,
                                          "unit": "GB/s", "frac": abytes / (us * 1e-6) / 1e9 / PEAK_HBM_GBS}
        out["adjoint_K64_M8_f32"] = res

    if want("large_rho"):
        # the benchmark workload at rho = R * mean(S^m): the cost term c/rho is
        # tiny next to theta, so active sets are large and the threshold search
        # does more passes (the regime where the candidate filter matters least)
        pr = inputs.balanced_sparse(dtype="f32")
        pr = dataclasses.replace(pr, rho=float(pr.R * np.mean(pr.S)))
        s = mam.solver_for(pr)
        s.init()
        s.iterate(10)
        n_it = 100
        dt = timed(lambda: s.iterate(n_it)) / n_it
        s.timing(True)
        s.iterate(50)
        col, n = s.timing_read()
        s.close()
        d = final_state(pr, 160, torch, mam)
        out["large_rho_K64_M32_f32"] = {"rho": pr.rho, "iterations": n_it, "ms_per_iter": dt * 1e3,
                                        "plan_entry_updates_per_s": pr.R * pr.T / dt, "column_kernel_ms": col / n,
                                        "column_kernel_GBs": algorithmic_bytes(pr) / (col / n * 1e-3) / 1e9,
                                        "state_after_160": d}
        log(f"rho = R * mean(S) = {pr.rho:.3g}: {dt * 1e3:.4f} ms/iter, column kernel {col / n:.4f} ms, "
            f"{d['rounds_per_column']:.2f} passes and {d['active_per_column']:.1f} active entries per column")

    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--cpu-measures", type=int, default=32)
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads")
    ap.add_argument("--extras", default="", help="comma-separated subset of the other workloads: " + ",".join(EXTRAS))
    args = ap.parse_args()
    only = [x for x in args.extras.split(",") if x] or None
    if only and not set(only) <= set(EXTRAS):
        ap.error(f"--extras: choose from {','.join(EXTRAS)}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2309_05315_amd import inputs

    # the paper's parallel CPU scheme runs first, in fresh processes started
    # before this process touches the GPU
    cpu_par = None
    if not args.no_cpu:
        p_cpu = inputs.balanced_sparse(dtype="f32")
        workers = max(1, min(16, len(os.sched_getaffinity(0)), p_cpu.M))
        cpu_par = cpu_baseline_parallel(p_cpu, workers)
        log(f"oracle, paper's parallel scheme on {workers} processes: {cpu_par['value']:.3e} entries/s")

    import torch
    from paper_2309_05315_amd import mam

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
    state32 = final_state(p32, args.warmup + args.steps, torch, mam)
    log(f"fp32 state after {state32['iterations']} iterations: {state32}")

    fp64 = None
    if not args.no_fp64:
        p64 = inputs.balanced_sparse(dtype="f64")
        dt64, pb64, col_ms64, _, sched64 = run_gpu(p64, args.steps, args.warmup, torch, mam)
        ab64 = algorithmic_bytes(p64)
        state64 = final_state(p64, args.warmup + args.steps, torch, mam)
        fp64 = {
            "value": entries * args.steps / dt64,
            "ms_per_step": dt64 / args.steps * 1e3,
            "column_kernel_ms": col_ms64,
            "achieved_GBs": ab64 / (col_ms64 * 1e-3) / 1e9,
            "fp32_speedup": dt64 / dt32,
            "barycenter_rel_l1_fp32_vs_fp64": float(np.abs(pb32 - pb64).sum() / np.abs(pb64).sum()),
            "barycenter_rel_max_fp32_vs_fp64": float(np.abs(pb32 - pb64).max() / np.abs(pb64).max()),
            "state": state64,
            "objective_rel_fp32_vs_fp64": abs(state32["W_hat"] - state64["W_hat"]) / abs(state64["W_hat"]),
        }
        log(f"fp64: {fp64['ms_per_step']:.4f} ms/iter; fp32/fp64 barycenter rel L1 "
            f"{fp64['barycenter_rel_l1_fp32_vs_fp64']:.3e}")

    copy = copy_ceiling(torch, mam)
    copy_gbs = copy["GBs"]
    log(f"device copy (library probe, 1 GiB, non-temporal, grid-stride): {copy_gbs:.0f} GB/s at "
        f"{copy['workgroups']} workgroups")

    traffic, traffic_note = None, "no counter record for this kernel source and schedule"
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        # counters apply only to the same kernel source launched the same way
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("schedule") == sched:
            traffic = tr.get("bytes_per_launch")
            traffic_note = (f"FETCH_SIZE + WRITE_SIZE of rocprofv3 runs stored in {os.path.relpath(TRAFFIC_FILE, ROOT)} "
                            "(taken on this kernel source and schedule, calibrated with the copy probe)")

    vs_oracle = error_vs_oracle(p32, torch, mam)
    log(f"fp32 vs the FP64 oracle after {vs_oracle['iterations']} iterations: {vs_oracle}")

    extras = None if args.no_extras else extra_workloads(torch, mam, inputs, log, only)

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
                   "S_drawn": sorted(int(x) for x in p32.S), "iterations": args.steps, "schedule": sched},
        "state": state32,
        "fp32_vs_oracle": vs_oracle,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "column_kernel", "algorithmic_bytes_per_launch": ab,
                     "traffic_source": traffic_note,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "copy_probe": copy,
                     "avg_launch_ms": col_ms32, "launches_timed": ncol},
        "fp64": fp64,
        "cpu_baseline": cpu,
        "cpu_baseline_parallel": cpu_par,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
