"""Full unbalanced extension (measure constraints sum_r pi_rs <= q_s, cost
shifted by eta) on the GPU vs the oracle's relaxed iteration, element by
element (MI355X only).  Tolerances 1e-10 (FP64 plans) and 1e-5 (FP32 plans)
relative, as for the other paths."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b, ord=1):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    if ord == 1:
        return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def shifted(p, eta):
    """The problem with the distances d = c - eta of the extension (rounded
    once to the storage precision, so both sides read the same values)."""
    c = p.cost - eta
    if p.dtype == "f32":
        c = c.astype(np.float32).astype(np.float64)
    return dataclasses.replace(p, cost=c)


def check(p, iters, **sched):
    say(f"case {p.name} {p.dtype} R={p.R} S={p.S} gamma={p.gamma} iters={iters} sched={sched}")
    cost = [p.cost_block(m) for m in range(p.M)]
    q = [p.q_block(m) for m in range(p.M)]
    ora = O.mam(cost, q, p.rho, p.gamma, iters, relaxed=True)
    s = mam.solver_for(p, relaxed=True, **sched)
    s.init()
    s.iterate(iters)
    pb = s.barycenter().cpu().numpy()
    th = s.plans()
    tol = TOL[p.dtype]
    e1, einf = rel(pb, ora["p_bar"]), rel(pb, ora["p_bar"], np.inf)
    eth = max(rel(a, b, np.inf) for a, b in zip(th, ora["theta"]))
    slack = min(float((ph.sum(axis=0) - qm).min()) for ph, qm in zip(ora["pi_hat"], q))
    say(f"  p_bar rel L1 {e1:.3e} max {einf:.3e}  theta rel max {eth:.3e}  oracle min column slack {slack:.3e}")
    assert e1 <= tol and einf <= tol
    if p.dtype == "f64":
        assert eth <= tol
    return s, ora, slack


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("eta,gamma", [(0.002, 0.2), (0.3, 0.05), (0.02, math.inf)])
def test_relaxed_short_path_matches_oracle(dtype, eta, gamma):
    masses = [0.7, 1.0, 1.3]
    p = shifted(inputs.tiny_problem(31, R=150, S=[40, 25, 33], dtype=dtype, masses=masses, gamma=gamma), eta)
    _, _, slack = check(p, 40)
    if eta <= 0.02:
        assert slack < -1e-6  # some columns keep part of their mass: the relaxation is active


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_relaxed_long_path_matches_oracle(dtype):
    p = shifted(inputs.tiny_problem(32, R=2300, S=[30, 22], dtype=dtype, masses=[0.8, 1.2], gamma=0.1), 0.0002)
    _, _, slack = check(p, 25, rows_per_tile=1024)
    assert slack < -1e-6


def test_relaxed_diagnostics_report_excess_only():
    p = shifted(inputs.tiny_problem(33, R=90, S=[20, 30], masses=[0.6, 1.4], gamma=0.2), 0.1)
    s = mam.solver_for(p, relaxed=True, diag=True)
    s.init()
    s.iterate(30)
    d = s.diagnostics()
    assert 0.0 <= d["meas_resid"] <= 1e-12


def test_relaxed_has_no_reverse_mode():
    p = shifted(inputs.tiny_problem(34, R=40, S=[10, 12], gamma=0.2), 0.1)
    s = mam.solver_for(p, relaxed=True)
    s.init()
    with pytest.raises(mam.MAMError):
        s.record(3)
