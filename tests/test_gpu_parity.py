"""HIP path vs the FP64 oracle, element by element (MI355X only).

Tolerances (relative): 1e-10 for FP64 plans, 1e-5 for FP32 plans, on the
barycenter (L1 and max norms), on every plan entry (max norm of the
difference over the max norm of the oracle's plans, per measure) and on the
marginals p^(m).  The oracle consumes exactly the (rounded) inputs the GPU
consumes.
"""
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


def run_gpu(p, iters, diag=False, cold=False, **sched):
    s = mam.solver_for(p, diag=diag, cold=cold, **sched)
    s.init()
    s.iterate(iters)
    pb = s.barycenter().cpu().numpy()
    out = {"p_bar": pb, "theta": s.plans(), "pm": s.marginals().cpu().numpy(), "solver": s}
    if diag:
        out["diag"] = s.diagnostics()
    return out


def check(p, iters, gate_theta=True, **sched):
    say(f"case {p.name} dtype={p.dtype} R={p.R} S={p.S[:4]}... iters={iters} sched={sched}")
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, iters)
    g = run_gpu(p, iters, **sched)
    tol = TOL[p.dtype]
    e1, einf = rel(g["p_bar"], ora["p_bar"]), rel(g["p_bar"], ora["p_bar"], np.inf)
    eth = max(rel(a, b, np.inf) for a, b in zip(g["theta"], ora["theta"]))
    say(f"  p_bar rel L1 {e1:.3e}  max {einf:.3e}  theta rel max {eth:.3e}")
    assert e1 <= tol and einf <= tol
    if gate_theta:
        assert eth <= tol
    epm = np.abs(g["pm"] - ora["pm"]).max() / np.abs(ora["pm"]).max()
    say(f"  marginals rel max {epm:.3e}")
    assert epm <= tol
    return g, ora


def test_gpu_present():
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    mam.lib()


def test_balanced_plain_full_run_fp64():
    """16x16 grid, M = 4, FP64, 200 iterations (Gaussian-tail weights down to ~1e-87)."""
    check(inputs.balanced_plain(), 200)


@pytest.mark.parametrize("R,S,dtype", [
    (1, [3, 2], "f64"), (5, [7, 1, 4], "f64"), (63, [9, 17], "f32"), (64, [40], "f64"),
    (65, [20, 30], "f32"), (200, [33, 12, 50], "f64"), (257, [31, 8], "f32"),
    (513, [40, 21], "f64"), (1000, [25, 19, 7], "f32"), (1024, [30, 30], "f64"),
    (1030, [17, 23], "f32"), (2049, [20, 11], "f64"), (4096, [24, 9], "f32"),
    (4099, [10, 13], "f64"), (5000, [6, 5], "f64"), (8192, [4, 3], "f32"),
])
def test_shapes_ragged(R, S, dtype):
    """Every column shape (threads per column x values per thread, vector and
    scalar tails), per-column costs, zero weights, uneven S^m."""
    p = inputs.tiny_problem(R + len(S), R=R, S=S, dtype=dtype, zero_frac=0.15, iters=12)
    check(p, 12)


@pytest.mark.parametrize("gamma,dtype", [(0.01, "f64"), (0.01, "f32"), (0.3, "f64"), (0.0, "f64")])
def test_unbalanced(gamma, dtype):
    p = inputs.unbalanced_dense(K=16, M=10, iters=60, gamma=gamma, dtype=dtype)
    g, ora = check(p, 60)
    if gamma > 0:
        assert ora["t"] < 1.0           # the damping branch is exercised


def test_unbalanced_damping_history():
    """t^k of every iteration equals the oracle's."""
    p = inputs.unbalanced_dense(K=8, M=5, gamma=0.01, dtype="f64")
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, 25, record=True)
    s = mam.solver_for(p, diag=True)
    s.init()
    ts = []
    for k in range(25):
        s.iterate(1)
        ts.append(s.diagnostics()["t"])
    np.testing.assert_allclose(ts, ora["hist"]["t"], rtol=1e-12)
    assert min(ts) < 1.0


@pytest.mark.parametrize("dtype,order", [("f64", 0), ("f32", 0), ("f32", 2)])
def test_indexed_sparse_quarter_scale(dtype, order):
    """Sparse supports (zero pixels removed) with the grid cost gathered by
    index, in measure-major and cost-block-major column order."""
    p = inputs.balanced_sparse(K=24, M=8, iters=40, dtype=dtype)
    check(p, 40, order=order)


@pytest.mark.parametrize("nt,nwg,remap", [
    (64, 1, -1), (64, 0, 1), (128, 7, -1), (256, 0, 0), (512, 3, 1), (1024, 0, 0), (256, 10000, -1),
])
def test_schedules(nt, nwg, remap):
    p = inputs.tiny_problem(77, R=900, S=[37, 5, 61, 12], dtype="f64", zero_frac=0.1, iters=15)
    check(p, 15, threads_per_column=nt, workgroups=nwg, xcd_remap=remap)


def test_bitwise_determinism():
    p = inputs.balanced_sparse(K=16, M=6, iters=30, dtype="f32")
    a = run_gpu(p, 30)
    b = run_gpu(p, 30)
    assert np.array_equal(a["p_bar"], b["p_bar"])
    for x, y in zip(a["theta"], b["theta"]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nt", [16, 256])
def test_bitwise_equal_across_schedules(dtype, nt):
    """Every pi_hat entry enters the marginals' row sums as its own
    fixed-point integer, so for one thread shape the iterate does not depend
    on how the columns are dealt to workgroups: workgroup count, team sweeps,
    column order, XCD mapping and columns in flight give the same plans,
    marginals and barycenter bit for bit."""
    p = inputs.balanced_sparse(K=16, M=6, iters=30, dtype=dtype)
    scheds = [dict(), dict(workgroups=7), dict(workgroups=333, team_size=4), dict(order=2, xcd_remap=1),
              dict(order=1, xcd_remap=-1, workgroups=64, team_size=16)]
    if nt == 256:
        scheds.append(dict(columns_in_flight=2))
    ref = None
    for sc in scheds:
        g = run_gpu(p, 30, threads_per_column=nt, **sc)
        say(f"case nt={nt} {dtype} sched={g['solver'].schedule()}")
        g["solver"].close()
        if ref is None:
            ref = g
            continue
        assert np.array_equal(g["p_bar"], ref["p_bar"]), sc
        assert np.array_equal(g["pm"], ref["pm"]), sc
        for x, y in zip(g["theta"], ref["theta"]):
            assert np.array_equal(x, y), sc


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_large_finite_gamma_is_bitwise_balanced(dtype):
    """A finite gamma at or above rho * max_k d_k leaves t = 1 in every
    iteration (Alg. 1, the damping of the unbalanced case), so the iterates
    equal the balanced ones bit for bit; the bound is taken from the oracle's
    d history with a wide margin for the GPU's own rounding."""
    import dataclasses
    p = inputs.balanced_sparse(K=16, M=5, iters=40, dtype=dtype)
    cost, q = blocks(p)
    hist = O.mam(cost, q, p.rho, math.inf, 40, record=True)["hist"]["d"]
    bound = 10.0 * p.rho * max(hist)
    say(f"case gamma=inf vs gamma={bound:.3e} dtype={dtype} R={p.R} M={p.M}")
    a = run_gpu(p, 40)
    b = run_gpu(dataclasses.replace(p, gamma=bound), 40)
    assert np.array_equal(a["p_bar"], b["p_bar"])
    for x, y in zip(a["theta"], b["theta"]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_unbalanced_mass_relation_per_iteration(dtype):
    """Every column of theta' is pi_hat - t b^(m) with pi_hat summing to q_s
    (Alg. 1, Prop. 3), so each measure's mass moves by
    sum_r p^(m),k+1 = sum q^(m) - t^k (sum_r p^k - sum_r p^(m),k), with t^k the
    damping of that iteration; checked on the device's own iterates."""
    p = inputs.tiny_problem(21, R=700, S=[40, 65, 33], masses=[0.7, 1.0, 1.3], gamma=0.05, dtype=dtype)
    s = mam.solver_for(p, diag=True)
    s.init()
    qsum = np.array([p.q_block(m).sum() for m in range(p.M)])
    tol = 1e-12 if dtype == "f64" else 1e-5
    ts = []
    for k in range(8):
        pm = s.marginals().cpu().numpy()
        pb = s.barycenter().cpu().numpy()
        s.iterate(1)
        t = s.diagnostics()["t"]
        ts.append(t)
        pm1 = s.marginals().cpu().numpy()
        want = qsum - t * (pb.sum() - pm.sum(axis=1))
        err = np.abs(pm1.sum(axis=1) - want).max() / qsum.max()
        assert err <= tol, (k, err)
    say(f"  t over 8 iterations: {[round(x, 4) for x in ts]}")
    assert min(ts) < 1.0  # the damped branch was taken


@pytest.mark.parametrize("gamma,kc", [(math.inf, 1), (0.05, 1), (math.inf, 4)])
def test_diagnostics_match_oracle(gamma, kc):
    """With kc = 4 the plain iterations walk the tables four columns per group
    step and the diagnostics iteration walks the same blocks one column at a
    time."""
    masses = None if math.isinf(gamma) else [0.7, 1.0, 1.3]
    p = inputs.tiny_problem(5, R=300, S=[40, 70, 25], masses=masses, gamma=gamma, dtype="f64")
    cost, q = blocks(p)
    k = 9
    prev = O.mam(cost, q, p.rho, p.gamma, k - 1)
    ora = O.mam(cost, q, p.rho, p.gamma, k)
    od = O.diagnostics(cost, q, ora["pi_hat"], ora["theta"], prev["theta"])
    g = run_gpu(p, k, diag=True, threads_per_column=64, columns_in_flight=kc)
    gd = g["diag"]
    assert gd["iterations"] == k
    assert rel(g["p_bar"], ora["p_bar"]) <= 1e-10
    assert gd["rounds_per_column"] >= 1.0 and gd["active_per_column"] >= 1.0
    assert abs(gd["W_hat"] - od["W_hat"]) <= 1e-10 * abs(od["W_hat"])
    assert abs(gd["dist_L"] - od["dist_L"]) <= 1e-8 * max(od["dist_L"], 1e-12)
    assert gd["meas_resid"] <= 1e-14 and od["meas_resid"] <= 1e-14
    assert abs(gd["dtheta_inf"] - od["dtheta_inf"]) <= 1e-10 * od["dtheta_inf"]
    np.testing.assert_allclose(gd["dp_norm"], np.linalg.norm(ora["p_bar"] - prev["p_bar"]), rtol=1e-8)
    np.testing.assert_allclose(gd["t"], ora["t"], rtol=1e-12)


@pytest.mark.parametrize("dtype,R,ld", [("f32", 7, 7), ("f32", 10, 13), ("f64", 5, 5), ("f64", 300, 301)])
def test_custom_start_with_unaligned_columns(dtype, R, ld):
    """A caller's theta^0 and plans whose column stride is not a multiple of
    the vector width (single-element copies and loads): results match the
    oracle, and the padding rows of theta are never written."""
    p = inputs.tiny_problem(60 + R, R=R, S=[6, 9], dtype=dtype)
    dt = torch.float32 if dtype == "f32" else torch.float64
    cost, q = blocks(p)
    rng = np.random.default_rng(R)
    th0 = [np.abs(rng.normal(size=(R, sm))) * 1e-2 for sm in p.S]
    if dtype == "f32":
        th0 = [x.astype(np.float32).astype(np.float64) for x in th0]
    ora = O.mam(cost, q, p.rho, p.gamma, 10, theta0=th0)
    if p.col_index is None:
        mode = mam.COST_SHARED
    elif np.array_equal(p.col_index, np.arange(p.T)):
        mode = mam.COST_PER_COLUMN
    else:
        mode = mam.COST_INDEXED
    s = mam.Solver(R, p.S, rho=p.rho, gamma=p.gamma, dtype=dt, cost_mode=mode, cost_ncols=p.cost_ncols,
                   ld=ld, cost_ld=ld)
    c = torch.full((p.cost_ncols, ld), 7.0, dtype=dt)
    c[:, :R] = torch.from_numpy(p.cost).to(dt)
    theta = torch.full((p.T, ld), 123.0, dtype=dt, device="cuda")
    idx = torch.from_numpy(p.col_index.astype(np.int32)).cuda() if mode == mam.COST_INDEXED else None
    s.bind(theta, c.cuda(), torch.from_numpy(p.q).to(dt).cuda(), idx)
    t0 = torch.full((p.T, ld), -5.0, dtype=dt)
    t0[:, :R] = torch.from_numpy(np.concatenate([x.T for x in th0])).to(dt)
    s.init(t0.cuda())
    s.iterate(10)
    say(f"case R={R} ld={ld} {dtype} schedule={s.schedule()}")
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= TOL[dtype]
    th = theta.cpu().numpy()
    assert np.all(th[:, R:] == 123.0)
    off = np.concatenate([[0], np.cumsum(p.S)])
    for m in range(p.M):
        assert rel(th[off[m]:off[m + 1], :R].T, ora["theta"][m], np.inf) <= TOL[dtype]


def test_custom_start_and_resume():
    """theta^0 given by the caller; iterate(a) then iterate(b) equals iterate(a+b)."""
    p = inputs.tiny_problem(8, R=128, S=[20, 30], dtype="f64")
    cost, q = blocks(p)
    rng = np.random.default_rng(3)
    th0 = [np.abs(rng.normal(size=(128, s))) * 1e-3 for s in p.S]
    ora = O.mam(cost, q, p.rho, p.gamma, 10, theta0=th0)
    s = mam.solver_for(p)
    t0 = torch.zeros_like(s.theta)
    t0[:, :128] = torch.from_numpy(np.concatenate([t.T for t in th0])).to(s.theta)
    s.init(t0)
    s.iterate(4)
    s.iterate(6)
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= 1e-10
    for a, b in zip(s.plans(), ora["theta"]):
        assert rel(a, b, np.inf) <= 1e-10


def test_edge_cases():
    # M = 1 (the barycenter of one measure), S^m = 1 columns, all-zero measure columns
    for p in (inputs.tiny_problem(1, R=50, S=[30], dtype="f64"),
              inputs.tiny_problem(2, R=70, S=[1, 1, 1], dtype="f64"),
              inputs.tiny_problem(3, R=33, S=[12, 9], dtype="f64", zero_frac=0.9)):
        check(p, 20)
    # zero iterations: the barycenter of theta^0 = q/R is (mass / R) everywhere
    p = inputs.tiny_problem(4, R=10, S=[3, 4], dtype="f64")
    g = run_gpu(p, 0)
    np.testing.assert_allclose(g["p_bar"], np.full(10, 0.1), rtol=1e-15)


def test_input_errors():
    p = inputs.tiny_problem(6, R=40, S=[5, 6], dtype="f64")
    s = mam.solver_for(p)
    q_bad = s.q.clone()
    q_bad[0] = q_bad[0] * 1.5                      # masses differ in balanced mode
    s.bind(s.theta, s.cost, q_bad)
    with pytest.raises(mam.MAMError) as e:
        s.init()
    assert e.value.status == "MAM_ENOTBALANCED"
    q_neg = s.q.clone()
    q_neg[1] = -q_neg[1]
    s.bind(s.theta, s.cost, q_neg)
    with pytest.raises(mam.MAMError) as e:
        s.init()
    assert e.value.status == "MAM_ENONFINITE"
    c_nan = s.cost.clone()
    c_nan[2, 3] = float("nan")
    s.bind(s.theta, c_nan, s.q.new_tensor(p.q))
    with pytest.raises(mam.MAMError) as e:
        s.init()
    assert e.value.status == "MAM_ENONFINITE"
    with pytest.raises(mam.MAMError):
        mam.Solver(40, [5, 6], dtype=torch.float64, cost_mode=mam.COST_PER_COLUMN).iterate(1)


def test_index_out_of_range_rejected():
    p = inputs.balanced_sparse(K=8, M=3, dtype="f64")
    s = mam.solver_for(p)
    bad = s.index.clone()
    bad[5] = p.cost.shape[0]
    s.bind(s.theta, s.cost, s.q, bad)
    with pytest.raises(mam.MAMError) as e:
        s.init()
    assert e.value.status == "MAM_ENONFINITE"


def test_cost_helper():
    # the squared distance is a sum of rounded squares in axis order on both
    # sides (no fused multiply-add), the max is exact and the division is
    # correctly rounded: equal bit for bit, also after rounding to FP32
    K = 12
    pts = inputs.grid_points(K)
    zeta = np.random.default_rng(1).uniform(0, 1, size=(37, 2))
    xi_t = torch.from_numpy(pts).cuda()
    z_t = torch.from_numpy(zeta).cuda()
    for norm in (False, True):
        ref = O.sq_euclid_cost(pts, zeta, normalize_max=norm)
        got = mam.cost_sq_euclid(xi_t, z_t, normalize_max=norm, dtype=torch.float64).cpu().numpy()
        np.testing.assert_array_equal(got.T, ref)
        g32 = mam.cost_sq_euclid(xi_t, z_t, normalize_max=norm, dtype=torch.float32, ld=K * K + 3)
        np.testing.assert_array_equal(g32[:, :K * K].cpu().numpy().T, ref.astype(np.float32))


@pytest.mark.parametrize("nt,kc", [(64, 1), (64, 2), (64, 4), (256, 2), (512, 4), (1024, 2)])
def test_columns_in_flight_and_warm_start(nt, kc):
    """Warm-started thresholds and any number of columns in flight give the
    same plans, bitwise, as cold starts one column at a time."""
    p = inputs.balanced_sparse(K=16, M=5, iters=25, dtype="f32")
    ref = run_gpu(p, 25, threads_per_column=64, columns_in_flight=1, cold=True)
    got = run_gpu(p, 25, threads_per_column=nt, columns_in_flight=kc)
    if nt == 64:
        assert np.array_equal(ref["p_bar"], got["p_bar"])
        for x, y in zip(ref["theta"], got["theta"]):
            assert np.array_equal(x, y)
    else:   # a different group width sums in a different order
        assert rel(got["p_bar"], ref["p_bar"]) <= 1e-6
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, 25)
    assert rel(got["p_bar"], ora["p_bar"]) <= TOL["f32"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_large_rho_regime(dtype):
    """rho = R * mean(S): c/rho is tiny, most entries of a column are active
    and the threshold search takes many rounds (the opposite regime of the
    benchmark workloads, where a column has one or two active entries)."""
    p = inputs.balanced_plain(K=12, M=3, dtype=dtype)
    p.rho = float(p.R * np.mean(p.S))
    g, _ = check(p, 25)
    s = mam.solver_for(p, diag=True)
    s.init()
    s.iterate(25)
    d = s.diagnostics()
    say(f"  rho={p.rho:.0f}: rounds/column {d['rounds_per_column']:.2f}, active/column {d['active_per_column']:.1f}")
    assert d["active_per_column"] > 10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("R,nt", [(1024, 64), (4096, 256), (4096, 1024)])
def test_threshold_ties_across_waves(dtype, R, nt):
    """Columns of R rows whose costs take four values only, plus one column
    of constant cost.  The first iteration starts from theta = q_s / R and
    b = 0, so w has long runs of exactly equal entries spread over every wave
    of a column (the constant column ties everywhere: its active set is the
    whole column).  The projection is unique however the ties fall, so the
    plans match the oracle entry by entry after one iteration and after
    fifteen, whichever waves hold the active entries.

    Plan tolerance.  In the constant column lambda comes from a sum of R
    values of w near -0.5, and pi_hat = w - lambda is only q_s / R: the
    rounding of that sum (at most about R u max|w| for the oracle's
    sequential prefix sums, u = 2^-53, |w| <= 1 here) is an absolute error of
    every plan entry of the column.  The plans are therefore gated at that
    bound relative to their largest entry when it exceeds the usual
    tolerance; the barycenter and the marginals keep the usual tolerance."""
    import dataclasses
    p = inputs.tiny_problem(41, R=R, S=[6, 5], dtype=dtype, masses=[1.0, 1.0])
    c = np.round(p.cost * 3.0) / 3.0
    c[0, :] = 0.5
    if dtype == "f32":
        c = c.astype(np.float32).astype(np.float64)
    p = dataclasses.replace(p, cost=np.ascontiguousarray(c))
    for iters in (1, 15):
        g, ora = check(p, iters, gate_theta=False, threads_per_column=nt)
        for a, b in zip(g["theta"], ora["theta"]):
            bound = 2.0 * R * 2.0 ** -53 / np.abs(b).max()
            assert rel(a, b, np.inf) <= max(TOL[dtype], bound)
        if iters == 1:
            # the constant column spreads its mass evenly over all rows (up to
            # the same rounding, cancelled down to q_s / R)
            np.testing.assert_allclose(np.asarray(g["theta"][0])[:, 0], p.q[0] / p.R, rtol=0, atol=1e-11)
