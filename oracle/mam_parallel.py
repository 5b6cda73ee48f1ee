"""Alg. 1 of the FP64 oracle run in the paper's parallel scheme.

TEST INFRASTRUCTURE ONLY.  Only the test suite and the scripts that write
stored reference values may import or run this module; the HIP library never
calls it and shares no code with it.

The paper parallelises MAM over measures: every process owns the plans of
some measures and runs Step 2 (and the row sums of Step 3) for them, and the
average p = sum_m a_m p^(m) of Step 1 is the gathering step between the
processes (Prop. 2 and the text after it; Sec. 6, where the measures are
dealt over the processors).  Here each worker process owns a group of
measures for the whole run; per iteration the main process sends the M x R
marginals and every worker advances its own plans with ``mam_step`` of
``mam_oracle`` restricted to its measures, then returns their new
marginals.  Every number is computed by the same numpy statements, on the
same data, as the one-process ``mam_oracle.mam``, so the results are equal
bit for bit (a test checks this); only the time is divided.

A worker builds its inputs itself from a picklable callable (for example a
``functools.partial`` of a generator), so no plan or cost block crosses a
process boundary.  The callable returns an object with ``R``, ``S``,
``rho``, ``gamma``, ``cost_block(m)`` and ``q_block(m)``.
"""
from __future__ import annotations

import multiprocessing as mp
from typing import Callable, Dict, List, Sequence

import numpy as np

from . import mam_oracle as O


def _worker(conn, build: Callable, measures: Sequence[int]):
    prob = build()
    R, S, M = prob.R, list(prob.S), len(prob.S)
    mine = list(measures)
    # placeholders for the other measures' plans and costs: mam_step reads
    # only their column counts and passes them through untouched
    theta: List[np.ndarray] = [np.empty((0, S[m])) for m in range(M)]
    cost: List[np.ndarray] = [np.empty((0, S[m])) for m in range(M)]
    q = [prob.q_block(m) for m in range(M)]
    for m in mine:
        cost[m] = np.asarray(prob.cost_block(m), dtype=np.float64)
        theta[m] = np.repeat((q[m] / R)[None, :], R, axis=0)     # theta^0 = q_s / R
    conn.send(O.marginals([theta[m] for m in mine]))            # Step 0, own rows
    while True:
        msg = conn.recv()
        if msg[0] == "stop":
            break
        _, pm, last = msg
        new_theta, pm_new, info = O.mam_step(theta, pm, cost, q, prob.rho, prob.gamma, chosen=mine)
        reply = {"pm": pm_new[mine], "t": info["t"], "d": info["d"]}
        if last:
            # the figures of the last iteration, measure by measure
            per = [O.diagnostics([cost[m]], [q[m]], [info["pi_hat"][m]], [new_theta[m]], [theta[m]])
                   for m in mine]
            reply["W"] = [x["W_hat"] for x in per]
            reply["meas_resid"] = [x["meas_resid"] for x in per]
            reply["dtheta_inf"] = [x["dtheta_inf"] for x in per]
            reply["pm_hat"] = O.marginals([info["pi_hat"][m] for m in mine])
        theta = new_theta
        conn.send(reply)
    conn.close()


def mam_parallel(build: Callable, iters: int, workers: int, log: Callable = None) -> Dict:
    """``iters`` iterations of Alg. 1 (M^k = all measures, theta^0 = q_s/R)
    on ``workers`` processes, measures dealt round robin.

    Returns p_bar (= sum_m a_m p^(m) of theta^K), pm, the last t, and the
    figures of the last iteration as ``mam_oracle.diagnostics`` defines
    them: W_hat = sum_m <c^(m), pi_hat^(m)>, dist_L(pi_hat), meas_resid,
    dtheta_inf; plus pm_hat, the row sums of pi_hat (M x R).
    """
    if iters < 1:
        raise ValueError("iters must be >= 1")
    prob = build()
    R, S, M = prob.R, list(prob.S), len(prob.S)
    workers = max(1, min(workers, M))
    groups = [list(range(w, M, workers)) for w in range(workers)]
    ctx = mp.get_context("spawn")
    conns, procs = [], []
    for g in groups:
        a, b = ctx.Pipe()
        pr = ctx.Process(target=_worker, args=(b, build, g), daemon=True)
        pr.start()
        conns.append(a)
        procs.append(pr)
    try:
        pm = np.zeros((M, R))
        for c, g in zip(conns, groups):
            pm[g] = c.recv()
        last = {}
        for k in range(iters):
            fin = k == iters - 1
            for c in conns:
                c.send(("step", pm, fin))
            pm_new = np.empty_like(pm)
            replies = []
            for c, g in zip(conns, groups):
                r = c.recv()
                pm_new[g] = r["pm"]
                replies.append(r)
            if fin:
                last = {"replies": replies}
            t, d = replies[0]["t"], replies[0]["d"]
            pm = pm_new
            if log and (k + 1) % 50 == 0:
                log(f"  iteration {k + 1}/{iters}: t={t:.6g} d={d:.6g}")
        W = [0.0] * M
        res = [0.0] * M
        dth = [0.0] * M
        pm_hat = np.empty((M, R))
        for r, g in zip(last["replies"], groups):
            for i, m in enumerate(g):
                W[m], res[m], dth[m] = r["W"][i], r["meas_resid"][i], r["dtheta_inf"][i]
            pm_hat[g] = r["pm_hat"]
        return {
            "p_bar": O.average(pm, S), "pm": pm, "t": t,
            # measure order, as diagnostics() sums and maximises them
            "W_hat": sum(W[m] for m in range(M)),
            "dist_L": O.dist_L_marginals(pm_hat, S),
            "meas_resid": max(res), "dtheta_inf": max(dth), "pm_hat": pm_hat,
        }
    finally:
        for c in conns:
            try:
                c.send(("stop",))
            except (BrokenPipeError, OSError):
                pass
        for pr in procs:
            pr.join(timeout=30)
            if pr.is_alive():
                pr.terminate()
