"""Long-column path (row tiles, candidate lists, per-column thresholds) vs
the FP64 oracle, element by element (MI355X only).

The path is forced on small problems (rows_per_tile = 1024 with R spanning
several tiles and a ragged last tile) so the oracle runs the same iterations
in seconds; R > 8192 takes it automatically.  A tiny candidate capacity
forces the fallback that recomputes a column from theta and c.  Tolerances
as for the short path: 1e-10 (FP64 plans) and 1e-5 (FP32 plans) relative.
"""
import dataclasses
import math
import sys

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


def run(p, iters, graph=0, **sched):
    s = mam.solver_for(p, **sched)
    sc = s.schedule()
    assert sc["rows_per_tile"] > 0, "the long-column path was not taken"
    if graph:
        s.graph(graph)
    s.init()
    s.iterate(iters)
    return s


def check(p, iters, **sched):
    say(f"case {p.name} {p.dtype} R={p.R} S={p.S} gamma={p.gamma} iters={iters} sched={sched}")
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, iters)
    s = run(p, iters, **sched)
    pb = s.barycenter().cpu().numpy()
    th = s.plans()
    tol = TOL[p.dtype]
    e1, einf = rel(pb, ora["p_bar"]), rel(pb, ora["p_bar"], np.inf)
    eth = max(rel(a, b, np.inf) for a, b in zip(th, ora["theta"]))
    say(f"  p_bar rel L1 {e1:.3e} max {einf:.3e}  theta rel max {eth:.3e}")
    assert e1 <= tol and einf <= tol
    if p.dtype == "f64":
        assert eth <= tol
    np.testing.assert_allclose(s.marginals().cpu().numpy(), ora["pm"], rtol=0,
                               atol=tol * np.abs(ora["pm"]).max() * 10)
    return s, ora


@pytest.mark.parametrize("R,S,dtype,shared", [
    (3000, [40, 25, 33], "f64", False),   # three tiles, ragged last one
    (2049, [17, 30], "f32", False),       # one row past two tiles
    (1024, [20, 20], "f64", True),        # exactly one tile, shared cost
    (4100, [12, 12], "f32", True),
    (2500, [7, 41, 3, 19], "f64", False),
])
def test_forced_long_path_matches_oracle(R, S, dtype, shared):
    p = inputs.tiny_problem(11, R=R, S=S, dtype=dtype, rho=1.0, shared=shared)
    check(p, 25, rows_per_tile=1024)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_unbalanced_long_path(dtype):
    p = inputs.tiny_problem(12, R=2200, S=[30, 22, 15], dtype=dtype, masses=[0.6, 1.0, 1.5], gamma=0.02)
    check(p, 30, rows_per_tile=1024)


@pytest.mark.parametrize("rho", [1.0, 200.0])
def test_candidate_overflow_falls_back_exactly(rho):
    # one slot per sub-tile overflows near every active set: those sub-tiles
    # are recomputed from theta and c in the threshold and write passes
    p = inputs.tiny_problem(13, R=2600, S=[24, 18], rho=rho)
    check(p, 20, rows_per_tile=1024, candidate_slots=1)


def test_large_rho_many_candidates():
    # rho = R * mean(S): large active sets, long candidate lists
    p = inputs.tiny_problem(14, R=2100, S=[16, 12], rho=2100.0 * 14)
    check(p, 15, rows_per_tile=1024)


def test_zero_weights_and_cold_start():
    p = inputs.tiny_problem(15, R=1500, S=[30, 26], zero_frac=0.4)
    check(p, 20, rows_per_tile=1024, cold=True)


@pytest.mark.parametrize("R", [8193, 12000])
def test_automatic_long_path_above_8192(R):
    p = inputs.tiny_problem(16, R=R, S=[9, 14], dtype="f32")
    s, _ = check(p, 12)
    assert s.schedule()["rows_per_tile"] == 4096


def test_bitwise_reproducible_and_graph_equals_eager():
    p = inputs.tiny_problem(17, R=3100, S=[35, 28], dtype="f32")
    a = run(p, 20, rows_per_tile=1024)
    b = run(p, 20, rows_per_tile=1024)
    g = run(p, 20, graph=5, rows_per_tile=1024)
    for x, y, z in zip(a.plans(), b.plans(), g.plans()):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)
    np.testing.assert_array_equal(a.barycenter().cpu().numpy(), g.barycenter().cpu().numpy())


def test_stopping_test_on_long_columns():
    p = inputs.tiny_problem(18, R=2300, S=[20, 31], rho=2.0)
    cost, q = blocks(p)
    s = mam.solver_for(p, rows_per_tile=1024)
    s.init()
    r = s.iterate_until(12, "dp", -1.0, 4)
    assert r["iterations"] == 12 and r["checks"] == 3
    ora = O.mam_until(cost, q, p.rho, 12, "dp", -1.0, 4)
    assert r["value"] == pytest.approx(ora["values"][-1], rel=1e-6)
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= 1e-10


def test_unsupported_on_long_columns():
    p = inputs.tiny_problem(19, R=1100, S=[10, 12])
    s = mam.solver_for(p, rows_per_tile=1024)
    s.init()
    with pytest.raises(mam.MAMError):
        s.record(3)
    with pytest.raises(mam.MAMError):
        s.set_bundles([0, 1])
    s = mam.solver_for(p, rows_per_tile=1024, sparse_store=True)
    s.init()
    with pytest.raises(mam.MAMError):
        s.iterate_until(4, "dtheta", 1e-3, 2)  # the sparse store keeps no dense copy to compare


DIAG_CASES = [
    ("three tiles, ragged last one", lambda: inputs.tiny_problem(21, R=3000, S=[40, 25, 33], dtype="f64"),
     dict(rows_per_tile=1024)),
    ("unbalanced, damped", lambda: inputs.tiny_problem(22, R=2200, S=[30, 22, 15], masses=[0.6, 1.0, 1.5],
                                                        gamma=0.02, dtype="f64"), dict(rows_per_tile=1024)),
    ("overflowing sub-tiles", lambda: inputs.tiny_problem(23, R=2600, S=[24, 18], rho=200.0, dtype="f64",
                                                          zero_frac=0.2), dict(rows_per_tile=1024, candidate_slots=1)),
    ("grid cost", lambda: inputs.free_support(seed=6, K=12, M=3, dtype="f64"), dict(rows_per_tile=1024, grid=True)),
]


@pytest.mark.parametrize("case", range(len(DIAG_CASES)))
@pytest.mark.parametrize("sparse", [False, True])
def test_long_diagnostics_match_oracle(case, sparse):
    """The figures of the last iteration on the long-column path: W_hat and the
    measure residual from the threshold kernel, ||theta^{k+1} - theta^k||_inf
    from the write kernel (dense store; NaN with the sparse store), dist_L from
    the marginals, against the oracle's."""
    name, gen, sched = DIAG_CASES[case]
    p = gen()
    say(f"case long diagnostics: {name} R={p.R} S={p.S} sparse={sparse}")
    cost, q = blocks(p)
    k = 9
    prev = O.mam(cost, q, p.rho, p.gamma, k - 1)
    ora = O.mam(cost, q, p.rho, p.gamma, k)
    od = O.diagnostics(cost, q, ora["pi_hat"], ora["theta"], prev["theta"])
    s = mam.solver_for(p, diag=True, sparse_store=sparse, **sched)
    assert s.schedule()["rows_per_tile"] > 0
    s.init()
    s.iterate(k)
    gd = s.diagnostics()
    say(f"  W_hat {gd['W_hat']:.12e} / {od['W_hat']:.12e}; dist_L {gd['dist_L']:.6e} / {od['dist_L']:.6e}; "
        f"resid {gd['meas_resid']:.1e} / {od['meas_resid']:.1e}; dtheta {gd['dtheta_inf']:.6e} / "
        f"{od['dtheta_inf']:.6e}; rounds {gd['rounds_per_column']:.3f} active {gd['active_per_column']:.3f}")
    assert gd["iterations"] == k
    assert abs(gd["W_hat"] - od["W_hat"]) <= 1e-10 * abs(od["W_hat"])
    assert abs(gd["dist_L"] - od["dist_L"]) <= 1e-8 * max(od["dist_L"], 1e-12)
    qmax = max(float(np.abs(x).max()) for x in q)
    assert gd["meas_resid"] <= 1e-12 * qmax and od["meas_resid"] <= 1e-12 * qmax
    if sparse:
        assert math.isnan(gd["dtheta_inf"])
    else:
        assert abs(gd["dtheta_inf"] - od["dtheta_inf"]) <= 1e-10 * od["dtheta_inf"]
    assert gd["rounds_per_column"] >= 1.0 and gd["active_per_column"] >= 1.0
    np.testing.assert_allclose(gd["dp_norm"], np.linalg.norm(ora["p_bar"] - prev["p_bar"]), rtol=1e-8)
    np.testing.assert_allclose(gd["t"], ora["t"], rtol=1e-12)
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= 1e-10


def test_theta_stopping_test_on_long_columns():
    """||theta^{k+1} - theta^k||_inf checked on the device every 3 iterations
    from the write kernel's maxima, against the oracle's run."""
    p = inputs.tiny_problem(24, R=2300, S=[20, 31], rho=2.0, dtype="f64")
    cost, q = blocks(p)
    ora = O.mam_until(cost, q, p.rho, 30, "dtheta", -1.0, 3)
    s = mam.solver_for(p, rows_per_tile=1024)
    s.init()
    r = s.iterate_until(30, "dtheta", -1.0, 3)
    assert r["iterations"] == 30 and r["checks"] == 10
    assert r["value"] == pytest.approx(ora["values"][-1], rel=1e-10)
    tol = float(np.median(ora["values"]))
    want = O.mam_until(cost, q, p.rho, 30, "dtheta", tol, 3)
    s.init()
    r = s.iterate_until(30, "dtheta", tol, 3)
    assert r["converged"] and r["iterations"] == want["iters"]
    assert rel(s.barycenter().cpu().numpy(), want["p_bar"]) <= 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_measure_sets_schedule_matches_oracle(dtype):
    # one shared cost and equal S^m: the M workgroups of a set take the same
    # (tile, column) units, one measure each, on one XCD
    p = inputs.tiny_problem(20, R=3000, S=[400, 400, 400], dtype=dtype, shared=True, rho=2.0)
    s, _ = check(p, 12, rows_per_tile=1024)
    nwg = s.schedule()["workgroups"]
    assert nwg % (8 * p.M) == 0, nwg


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("rows", [0, 1024])
def test_grid_cost_matches_oracle(dtype, rows):
    # free-support problem of 3 nested-ellipse 12x12 images: R = 34^2 grid
    # points; the kernels form the cost from the grid and the pixel centres,
    # the oracle reads it from the points in FP64 (rounded to the dtype)
    p = inputs.free_support(seed=3, K=12, M=3, dtype=dtype)
    sched = {"grid": True}
    if rows:
        sched["rows_per_tile"] = rows
    check(p, 20, **sched)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("rows", [1024, 4096])
def test_grid_cost_equals_stored_cost(dtype, rows):
    # the same problem with the cost stored (built on the device from the
    # points) and formed in the kernels: both evaluate each cost entry as the
    # rounded sum of rounded squares, so every iterate is identical bit for bit
    p = inputs.free_support(seed=4, K=10, M=4, dtype=dtype)
    a = run(p, 15, grid=True, rows_per_tile=rows)
    b = run(p, 15, rows_per_tile=rows)
    for x, y in zip(a.plans(), b.plans()):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.barycenter().cpu().numpy(), b.barycenter().cpu().numpy())


SPARSE_CASES = [
    ("f64 three tiles", lambda: inputs.tiny_problem(11, R=3000, S=[40, 25, 33], dtype="f64", rho=1.0),
     dict(rows_per_tile=1024)),
    ("f32 one row past two tiles", lambda: inputs.tiny_problem(12, R=2049, S=[17, 30], dtype="f32"),
     dict(rows_per_tile=1024)),
    ("overflowing sub-tiles", lambda: inputs.tiny_problem(13, R=2600, S=[24, 18], rho=200.0),
     dict(rows_per_tile=1024, candidate_slots=1)),
    ("unbalanced", lambda: inputs.tiny_problem(12, R=2200, S=[30, 22, 15], masses=[0.6, 1.0, 1.5], gamma=0.02),
     dict(rows_per_tile=1024)),
    ("grid cost f32", lambda: inputs.free_support(seed=4, K=10, M=4, dtype="f32"),
     dict(rows_per_tile=1024, grid=True)),
    ("grid cost f64, 16 values per thread", lambda: inputs.free_support(seed=5, K=12, M=3, dtype="f64"),
     dict(rows_per_tile=4096, grid=True)),
    ("automatic above 8192 rows", lambda: inputs.tiny_problem(16, R=8193, S=[9, 14], dtype="f32"), {}),
    ("relaxed measure constraints", lambda: shifted(
        inputs.tiny_problem(32, R=2300, S=[30, 22], masses=[0.8, 1.2], gamma=0.1), 0.0002),
     dict(rows_per_tile=1024, relaxed=True)),
]


def shifted(p, eta):
    """The relaxed extension's distances d = c - eta (FP64 problem)."""
    return dataclasses.replace(p, cost=p.cost - eta)


@pytest.mark.parametrize("case", range(len(SPARSE_CASES)))
def test_sparse_store_equals_dense(case):
    """The sparse store (plans held as -b plus the entries above lambda between
    the iterations of a call) gives the dense path's plans, marginals and
    barycenter bit for bit after every call: plain runs, graph replay, a run
    with a stopping test, a re-initialisation and the support step."""
    name, gen, sched = SPARSE_CASES[case]
    p = gen()
    say(f"case sparse store: {name} R={p.R} S={p.S} {p.dtype} sched={sched}")
    sd = mam.solver_for(p, **sched)
    ss = mam.solver_for(p, sparse_store=True, **sched)
    assert ss.schedule()["rows_per_tile"] > 0

    def same(tag):
        for x, y in zip(sd.plans(), ss.plans()):
            np.testing.assert_array_equal(x, y, err_msg=tag)
        np.testing.assert_array_equal(sd.marginals().cpu().numpy(), ss.marginals().cpu().numpy(), err_msg=tag)
        np.testing.assert_array_equal(sd.barycenter().cpu().numpy(), ss.barycenter().cpu().numpy(), err_msg=tag)

    for s in (sd, ss):
        s.init()
        s.iterate(7)
    same("after 7 iterations")
    for s in (sd, ss):
        s.iterate(1)
        s.iterate(0)
    same("after 1 + 0 more")
    for s in (sd, ss):
        s.graph(3)
        s.iterate(7)
        s.graph(0)
    same("after 7 with graph replay")
    rd = sd.iterate_until(12, "dp", -1.0, 5)
    rs = ss.iterate_until(12, "dp", -1.0, 5)
    assert rd == rs
    same("after a run with a stopping test")
    for s in (sd, ss):
        s.init()
        s.iterate(3)
    same("after a re-initialisation")
    rng = np.random.default_rng(0)
    zeta = torch.from_numpy(rng.normal(size=(p.T, 2))).cuda()
    xi0 = rng.normal(size=(p.R, 2))
    out = [s.support_update([1.0 / p.M] * p.M, zeta, torch.from_numpy(xi0.copy()).cuda()) for s in (sd, ss)]
    np.testing.assert_array_equal(out[0][0].cpu().numpy(), out[1][0].cpu().numpy())
    np.testing.assert_array_equal(out[0][1].cpu().numpy(), out[1][1].cpu().numpy())
    same("after the support step")
    # and against the oracle: a fresh start, 3 iterations and the support
    # step's own iteration
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, 4, relaxed=sched.get("relaxed", False))
    pb = ss.barycenter().cpu().numpy()
    assert rel(pb, ora["p_bar"]) <= TOL[p.dtype]
