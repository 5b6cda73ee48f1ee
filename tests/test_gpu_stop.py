"""On-device stopping tests (Sec. 5, stopping criteria) vs the oracle's run
with the same test (MI355X only).

The stopping iteration is an integer decided by a floating-point value, so
every tolerance below is placed between two checked values of the oracle's
run with a relative margin far above the GPU/oracle rounding difference; the
iteration count must then match exactly, and the plans and barycenter at
that iteration match to 1e-10 (FP64) / 1e-5 (FP32) relative.  On the line
problems with gamma = 0 the plans reach diag(q^(m)) after one iteration, so
the stop comes at iteration 2 with a value at rounding level (closed form).
"""
import math
import sys
import time

import numpy as np
import pytest
import torch

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def rel(a, b, ord=1):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    if ord == 1:
        return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def separated_tol(values, margin, floor):
    """A tolerance that every check before index i exceeds and check i meets,
    each by a relative margin, with values[i] >= floor * values[0] (below
    that the value is mostly rounding); i is the latest such index short of
    the last few checks (so the run stops well before max_iters), or None."""
    best = None
    for i in range(1, len(values) - 4):
        if floor * values[0] <= values[i] < min(values[:i]) * (1 - margin) ** 2 * (1 - 1e-12):
            best = i
    if best is None:
        return None, None
    hi = min(values[:best])
    tol = math.sqrt(hi * values[best])
    assert values[best] <= tol * (1 - margin) and hi >= tol * (1 + margin)
    return best, tol


def run_until(p, max_iters, test, tol, every, graph=0, **sched):
    s = mam.solver_for(p, **sched)
    if graph:
        s.graph(graph)
    s.init()
    r = s.iterate_until(max_iters, test, tol, every)
    return s, r


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("test", ["dtheta", "dp"])
@pytest.mark.parametrize("every", [1, 2, 3])
def test_gamma_zero_line_closed_form(dtype, test, every):
    p = inputs.line_problem(0, R=7, M=3, dtype=dtype, rho=0.5, gamma=0.0)
    say(f"case line R=7 M=3 {dtype} {test} every={every}")
    cost, q = blocks(p)
    ora = O.mam_until(cost, q, p.rho, 40, test, 1e-15, every, gamma=0.0)
    s, r = run_until(p, 40, test, 1e-15, every)
    expect = max(2, every)
    assert ora["iters"] == expect
    assert r["iterations"] == expect and r["converged"] and r["checks"] == expect // every
    assert 0.0 <= r["value"] <= 1e-16
    for th, qm in zip(s.plans(), q):
        np.testing.assert_allclose(th, np.diag(qm), rtol=0, atol=1e-16)


def test_gamma_zero_line_dist_closed_form():
    p = inputs.line_problem(2, R=7, M=3, rho=0.5, gamma=0.0)
    cost, q = blocks(p)
    a = np.array([1.0 / s for s in p.S])
    a /= a.sum()
    ph = sum(am * qm for am, qm in zip(a, q))
    dist = math.sqrt(sum(float(((ph - qm) ** 2).sum()) / s for qm, s in zip(q, p.S)))
    s, r = run_until(p, 6, "dist", dist * (1 - 1e-9), 2)
    assert r["iterations"] == 6 and not r["converged"] and r["checks"] == 3
    assert r["value"] == pytest.approx(dist, rel=1e-12)
    s, r = run_until(p, 6, "dist", dist * (1 + 1e-9), 2)
    assert r["iterations"] == 2 and r["converged"]


CASES = [
    ("f64", inputs.tiny_problem, dict(seed=1, R=40, S=[30, 50, 20], rho=2.0), math.inf),
    ("f64", inputs.tiny_problem, dict(seed=2, R=300, S=[120, 90], rho=1.0, shared=False), math.inf),
    ("f64", inputs.tiny_problem, dict(seed=3, R=64, S=[64, 64, 64], rho=4.0, shared=True), math.inf),
    ("f64", inputs.tiny_problem, dict(seed=4, R=50, S=[40, 30], rho=2.0, masses=[0.7, 1.3]), 0.05),
    ("f32", inputs.tiny_problem, dict(seed=5, R=128, S=[100, 60], rho=2.0), math.inf),
]


@pytest.mark.parametrize("graph", [0, 6])
@pytest.mark.parametrize("test", ["dtheta", "dp", "dist"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_stop_iteration_matches_oracle(case, test, graph):
    dtype, gen, kw, gamma = CASES[case]
    p = gen(dtype=dtype, gamma=gamma, **kw)
    every = 3
    N = 240
    say(f"case {p.name} {dtype} gamma={gamma} test={test} graph={graph}")
    cost, q = blocks(p)
    ref = O.mam_until(cost, q, p.rho, N, test, -1.0, every, gamma=gamma)
    margin, floor = (1e-4, 1e-8) if dtype == "f64" else (5e-3, 1e-3)
    vtol = 1e-6 if dtype == "f64" else 1e-3
    i, tol = separated_tol(ref["values"], margin, floor)
    if i is None:
        # no check falls clearly below all earlier ones (dist_L of an
        # unbalanced run settles at a positive value): the run never stops
        assert not math.isinf(gamma)
        s, r = run_until(p, N, test, min(ref["values"]) * 0.5, every, graph=graph)
        assert not r["converged"] and r["iterations"] == N and r["checks"] == N // every
        assert r["value"] == pytest.approx(ref["values"][-1], rel=vtol)
        return
    ora = O.mam_until(cost, q, p.rho, N, test, tol, every, gamma=gamma)
    assert ora["iters"] == (i + 1) * every
    s, r = run_until(p, N, test, tol, every, graph=graph)
    say(f"  stop at {r['iterations']} (oracle {ora['iters']}), value {r['value']:.6e} vs {ref['values'][i]:.6e}")
    assert r["converged"] and r["iterations"] == ora["iters"] and r["checks"] == i + 1
    assert r["value"] == pytest.approx(ref["values"][i], rel=vtol)
    t = TOL[dtype]
    pb = s.barycenter().cpu().numpy()
    assert rel(pb, ora["p_bar"]) <= t and rel(pb, ora["p_bar"], np.inf) <= t
    assert max(rel(a, b, np.inf) for a, b in zip(s.plans(), ora["theta"])) <= t
    # the run continues from the stopped iterate
    s.iterate(5)
    cont = O.mam(cost, q, p.rho, gamma, ora["iters"] + 5)
    pb = s.barycenter().cpu().numpy()
    assert rel(pb, cont["p_bar"]) <= t


@pytest.mark.parametrize("test", ["dp", "dist", "dtheta"])
def test_never_stopping_equals_plain_run(test):
    p = inputs.tiny_problem(6, R=200, S=[80, 70, 60], rho=2.0)
    plain = mam.solver_for(p)
    plain.init()
    plain.iterate(10)
    s, r = run_until(p, 10, test, -1.0, 3)
    assert r["iterations"] == 10 and not r["converged"] and r["checks"] == 3
    for a, b in zip(s.plans(), plain.plans()):
        if test == "dtheta":
            # the check iterations use the diagnostics instance of the column kernel
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-15 * np.abs(b).max())
        else:
            np.testing.assert_array_equal(a, b)
    if test != "dtheta":
        np.testing.assert_array_equal(s.barycenter().cpu().numpy(), plain.barycenter().cpu().numpy())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_dtheta_is_the_change_of_the_stored_plans(dtype):
    """The device's ||theta^{k+1} - theta^k||_inf is the largest change of the
    stored plans (a difference of two floats is exact in double): equal bit
    for bit to the same maximum taken on the host from the plans read back
    before and after the iteration, at several iterations of a run."""
    p = inputs.tiny_problem(11, R=500, S=[120, 75, 200], rho=2.0, zero_frac=0.1, dtype=dtype)
    s = mam.solver_for(p, diag=True)
    s.init()
    say(f"case {p.name} {dtype}")
    for k in (1, 4, 20):
        before = s.plans()
        s.iterate(1)
        after = s.plans()
        d = s.diagnostics()
        host = max(float(np.abs(a - b).max()) for a, b in zip(after, before))
        say(f"  iteration {d['iterations']}: device {d['dtheta_inf']:.9e} host {host:.9e}")
        assert d["dtheta_inf"] == host
        s.iterate(k)


@pytest.mark.parametrize("graph", [0, 6])
def test_fp32_dtheta_stop_is_the_first_check_below_tol(graph):
    """FP32 plans, the ||theta^{k+1} - theta^k||_inf test: the run stops at
    the first check whose change of the stored plans, measured on the host
    from a plain run's plans, is <= tol, and its plans equal that run's."""
    p = inputs.tiny_problem(12, R=128, S=[100, 60], rho=2.0, dtype="f32")
    every, N = 3, 120
    plain = mam.solver_for(p)
    plain.init()
    vals, plans_at = [], {}
    prev = plain.plans()
    for j in range(1, N + 1):
        plain.iterate(1)
        cur = plain.plans()
        if j % every == 0:
            vals.append(max(float(np.abs(a - b).max()) for a, b in zip(cur, prev)))
            plans_at[j] = cur
        prev = cur
    plain.close()
    # a tolerance between a check and every check before it, with a margin
    # far above the difference the check iterations' kernel instance makes
    i, tol = separated_tol(vals, 5e-3, 1e-3)
    assert i is not None
    s, r = run_until(p, N, "dtheta", tol, every, graph=graph)
    say(f"  FP32 dtheta stop: {r['iterations']} (host {(i + 1) * every}), value {r['value']:.6e} vs {vals[i]:.6e}")
    assert r["converged"] and r["iterations"] == (i + 1) * every and r["checks"] == i + 1
    assert r["value"] == pytest.approx(vals[i], rel=1e-6)
    for a, b in zip(s.plans(), plans_at[r["iterations"]]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-6 * np.abs(b).max())


def test_first_check_and_empty_run():
    p = inputs.tiny_problem(7, R=50, S=[30, 20])
    s, r = run_until(p, 100, "dp", math.inf, 4)
    assert r["iterations"] == 4 and r["converged"] and r["checks"] == 1
    ora = O.mam(*blocks(p), p.rho, p.gamma, 4)
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= 1e-10
    r = s.iterate_until(0, "dp", 1.0, 1)
    assert r["iterations"] == 0 and r["checks"] == 0 and not r["converged"] and math.isnan(r["value"])
    r = s.iterate_until(3, "dp", 1.0, 5)  # no check falls inside the run
    assert r["iterations"] == 3 and r["checks"] == 0 and not r["converged"]


def test_diagnostics_after_theta_stop():
    p = inputs.tiny_problem(8, R=60, S=[40, 50], rho=2.0)
    s = mam.solver_for(p, diag=True)
    s.init()
    r = s.iterate_until(50, "dtheta", math.inf, 5)
    assert r["iterations"] == 5
    d = s.diagnostics()
    assert d["iterations"] == 5 and d["dtheta_inf"] == r["value"]


def test_errors():
    p = inputs.tiny_problem(9, R=20, S=[10, 12])
    s = mam.solver_for(p)
    with pytest.raises(mam.MAMError):
        s.iterate_until(5, "dp", 1e-3, 1)  # before init
    s.init()
    for args in [(5, "dp", 1e-3, 0), (5, "dp", float("nan"), 1), (-1, "dp", 1e-3, 1)]:
        with pytest.raises(mam.MAMError):
            s.iterate_until(*args)
    with pytest.raises(ValueError):
        s.iterate_until(5, "nope", 1e-3, 1)


@pytest.mark.parametrize("graph", [0, 10])
def test_full_size_early_exit(graph):
    """64x64 grid, 32 thresholded measures, FP32: a run told to stop at the
    first check (tol = inf) stops there and equals a plain run of that many
    iterations; a run that never stops equals the plain run; and the launches
    enqueued after the stop cost far less than the iterations they replace."""
    p = inputs.balanced_sparse(dtype="f32")
    say(f"case balanced_sparse f32 graph={graph}")
    plain = mam.solver_for(p)
    plain.init()
    plain.iterate(10)
    torch.cuda.synchronize()
    ref = plain.plans()
    pb_ref = plain.barycenter().cpu().numpy()
    plain.close()
    del plain
    s = mam.solver_for(p)
    if graph:
        s.graph(graph)
    s.init()
    r = s.iterate_until(10, "dp", -1.0, 5)
    assert r["iterations"] == 10 and r["checks"] == 2 and not r["converged"]
    np.testing.assert_array_equal(s.barycenter().cpu().numpy(), pb_ref)
    th = s.plans()
    for m in range(0, p.M, 7):
        np.testing.assert_array_equal(th[m], ref[m])
    s.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.iterate_until(20000, "dp", math.inf, 10)
    el = time.perf_counter() - t0
    say(f"  stop after {r['iterations']} of at most 20000 iterations in {el * 1e3:.1f} ms")
    assert r["iterations"] == 10 and r["converged"]
    assert el < 0.5  # 20000 iterations would take about 15 s
    np.testing.assert_array_equal(s.barycenter().cpu().numpy(), pb_ref)
