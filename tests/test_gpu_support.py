"""Support step (Prop. 4) and the alternation of Alg. 2 on the GPU vs the
FP64 oracle (MI355X only).

The GPU call runs one more iteration and then forms the support from that
iteration's projected plans; the oracle runs the same number of iterations
and applies its closed form to its pi_hat.  FP64 plans: the masses agree to
1e-10 of the largest and the points to 1e-9 of the points' range on rows
above 1e-6 of the largest mass; FP32 plans: 1e-5 and 1e-4 on rows above 1%
of it (the plans themselves agree to 1e-5 relative).  A point is a quotient
of two sums, so on rows with almost no mass it is set by rounding.  At the
full free-support size, sampled rows are rebuilt on the host from the plans
and marginals read back, in FP64, and must agree to 1e-12 relative.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-10, 1e-9), "f32": (1e-5, 1e-4)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def compare(p, xi_gpu, mass_gpu, ora, xi0, span):
    mtol, xtol = TOL[p.dtype]
    mo, xo = ora["mass"], ora["xi"]
    em = np.abs(mass_gpu - mo).max() / mo.max()
    rows = mo > (1e-2 if p.dtype == "f32" else 1e-6) * mo.max()
    ex = np.abs(xi_gpu[rows] - xo[rows]).max() / span
    say(f"  mass max err {em:.2e}, points max err {ex:.2e} on {rows.sum()} of {p.R} rows")
    assert em <= mtol and ex <= xtol
    # rows without mass on the GPU keep their points exactly
    none = mass_gpu <= 0
    np.testing.assert_array_equal(xi_gpu[none], xi0[none])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("rows", [0, 1024])
def test_support_step_matches_oracle(dtype, dim, rows):
    R = 2500 if rows else 300
    p = inputs.tiny_problem(31 + dim, R=R, S=[37, 52, 29], dtype=dtype, rho=2.0)
    say(f"case support R={R} dtype={dtype} dim={dim} rows_per_tile={rows}")
    rng = np.random.default_rng(dim)
    zeta = rng.normal(size=(p.T, dim))
    xi0 = rng.normal(size=(p.R, dim))
    alpha = np.array([0.2, 0.5, 0.3])
    K = 6
    sched = {"rows_per_tile": rows} if rows else {}
    s = mam.solver_for(p, **sched)
    s.init()
    s.iterate(K - 1)
    xi = torch.from_numpy(xi0.copy()).cuda()
    z = torch.from_numpy(zeta).cuda()
    xi, mass = s.support_update(alpha, z, xi)
    cost, q = blocks(p)
    run = O.mam(cost, q, p.rho, p.gamma, K)
    off = np.concatenate([[0], np.cumsum(p.S)])
    zb = [zeta[off[m]:off[m + 1]] for m in range(p.M)]
    ora = O.support_update(run["pi_hat"], zb, alpha, xi0)
    compare(p, xi.cpu().numpy(), mass.cpu().numpy(), ora, xi0, np.ptp(zeta))
    # the call ran the K-th iteration: the barycenter is the oracle's after K
    pb = s.barycenter().cpu().numpy()
    assert np.abs(pb - run["p_bar"]).sum() / np.abs(run["p_bar"]).sum() <= TOL[dtype][0]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_support_step_with_sparse_store_equals_dense(dtype):
    """With the sparse store the plans live as -b plus their patches between
    iterations; the support step writes them back before reading them, so
    points, masses and the plans themselves equal the dense run bit for bit,
    over two calls in a row."""
    p = inputs.tiny_problem(35, R=2600, S=[37, 52, 29], dtype=dtype, rho=2.0)
    rng = np.random.default_rng(7)
    zeta = torch.from_numpy(rng.normal(size=(p.T, 2))).cuda()
    xi0 = rng.normal(size=(p.R, 2))
    alpha = [0.2, 0.5, 0.3]
    out = []
    for sparse in (False, True):
        say(f"case support R={p.R} dtype={dtype} rows_per_tile=1024 sparse_store={sparse}")
        s = mam.solver_for(p, rows_per_tile=1024, sparse_store=sparse)
        s.init()
        s.iterate(3)
        xi = torch.from_numpy(xi0.copy()).cuda()
        res = []
        for _ in range(2):
            xi, mass = s.support_update(alpha, zeta, xi)
            s.iterate(2)
            res.append((xi.cpu().numpy().copy(), mass.cpu().numpy().copy()))
        out.append((res, [x.copy() for x in s.plans()], s.barycenter().cpu().numpy()))
        s.close()
    (ra, pa, ba), (rb, pb, bb) = out
    for (xa, ma), (xb, mb) in zip(ra, rb):
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ma, mb)
    for x, y in zip(pa, pb):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(ba, bb)


def test_support_step_is_reproducible_and_keeps_massless_rows():
    # zero weights leave whole rows without mass after the first iteration
    p = inputs.tiny_problem(40, R=200, S=[30, 25], zero_frac=0.5, rho=0.05)
    rng = np.random.default_rng(1)
    zeta = torch.from_numpy(rng.normal(size=(p.T, 2))).cuda()
    xi0 = rng.normal(size=(p.R, 2))
    out = []
    for _ in range(2):
        s = mam.solver_for(p)
        s.init()
        xi, mass = s.support_update([0.5, 0.5], zeta, torch.from_numpy(xi0.copy()).cuda())
        out.append((xi.cpu().numpy(), mass.cpu().numpy()))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    cost, q = blocks(p)
    run = O.mam(cost, q, p.rho, p.gamma, 1)
    zb = [zeta.cpu().numpy()[:30], zeta.cpu().numpy()[30:]]
    ora = O.support_update(run["pi_hat"], zb, [0.5, 0.5], xi0)
    compare(p, out[0][0], out[0][1], ora, xi0, float(zeta.max() - zeta.min()))
    say(f"  rows without mass: {(out[0][1] <= 0).sum()}")


@pytest.mark.parametrize("rows", [0, 1024])
def test_alternation_matches_oracle(rows):
    """Alg. 2: the cost alpha_m/2 ||xi - zeta||^2 rebuilt on the device from the
    new points each round, Alg. 1 continued on it, then the support step."""
    rng = np.random.default_rng(5)
    R, S = (1500, [40, 35]) if rows else (120, [40, 35])
    T = sum(S)
    xi0 = rng.uniform(0, 1, size=(R, 2))
    zeta = rng.uniform(0, 1, size=(T, 2))
    q = [rng.uniform(0.1, 1, size=s) for s in S]
    q = [v / v.sum() for v in q]
    alpha = np.array([0.4, 0.6])
    rho, outer, inner = 0.5, 3, 4
    say(f"case alternation R={R} rows_per_tile={rows}")
    sched = {"rows_per_tile": rows} if rows else {}
    s = mam.Solver(R, S, rho=rho, dtype=torch.float64, cost_mode=mam.COST_PER_COLUMN, **sched)
    theta = torch.zeros(T, s.ld, dtype=torch.float64, device="cuda")
    cost = torch.zeros(T, s.cost_ld, dtype=torch.float64, device="cuda")
    z = torch.from_numpy(zeta).cuda()
    xi = torch.from_numpy(xi0.copy()).cuda()
    col_alpha = torch.from_numpy(np.repeat(alpha, S)).cuda()[:, None]

    def build_cost():
        c = mam.cost_sq_euclid(xi, z, dtype=torch.float64)      # (T, R): column j's cost
        cost[:, :R] = 0.5 * col_alpha * c

    build_cost()
    s.bind(theta, cost, torch.from_numpy(np.concatenate(q)).cuda())
    s.init()
    got, masses = [], []
    for k in range(outer):
        if k:
            build_cost()
        s.iterate(inner - 1)
        xi, mass = s.support_update(alpha, z, xi)
        got.append(xi.cpu().numpy().copy())
        masses.append(mass.cpu().numpy())
    off = np.concatenate([[0], np.cumsum(S)])
    ora = O.free_support_alternation(xi0, [zeta[off[m]:off[m + 1]] for m in range(2)], q, alpha, rho,
                                     outer=outer, inner=inner)
    for k in range(outer):
        rows = masses[k] > 1e-6 * masses[k].max()
        err = np.abs(got[k][rows] - ora["xi"][k][rows]).max()
        say(f"  round {k}: max |xi - oracle| {err:.2e} on {rows.sum()} of {R} rows")
        assert err <= 1e-8


def test_full_size_free_support_sampled_rows():
    """349,281 support points, 10 images of 60x60, FP32 plans (50 GB): 40
    sampled rows rebuilt on the host from the plans and the marginals the
    iteration started from; the masses sum to sum_m alpha_m sum_s q_s."""
    p = inputs.free_support(dtype="f32")
    say(f"case free_support_K60_M10 support step, R={p.R} T={p.T}")
    s = mam.solver_for(p, grid=True)
    s.init()
    s.iterate(4)
    pm = s.marginals().cpu().numpy()
    pbar = s.barycenter().cpu().numpy()
    zeta = torch.from_numpy(np.tile(p.zeta, (p.M, 1))).cuda()
    xi0 = torch.from_numpy(p.xi.copy()).cuda()
    alpha = np.full(p.M, 1.0 / p.M)
    torch.cuda.synchronize()
    xi, mass = s.support_update(alpha, zeta, xi0)
    torch.cuda.synchronize()
    mass = mass.cpu().numpy()
    xi = xi.cpu().numpy()
    qsum = sum(alpha[m] * float(p.q_block(m).astype(np.float64).sum()) for m in range(p.M))
    say(f"  sum of masses {mass.sum():.9f} (expected {qsum:.9f}); rows with mass {(mass > 0).sum()}")
    assert abs(mass.sum() - qsum) <= 1e-5 * qsum
    # rows rebuilt on the host: pi_hat = theta' + b (t = 1 with gamma = inf), an
    # entry equal to -b in FP32 counting as 0
    rng = np.random.default_rng(0)
    heavy = np.argsort(mass)[-20:]
    rows = np.concatenate([heavy, rng.choice(p.R, 20, replace=False)])
    S = p.S[0]
    th = s.theta[:, torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)  # (T, n)
    for i, r in enumerate(rows):
        num, den = np.zeros(2), 0.0
        for m in range(p.M):
            b = 1.0 * (pbar[r] - pm[m, r]) / S
            col = th[m * S:(m + 1) * S, i]
            pi = np.where(col.astype(np.float32) == np.float32(-b), 0.0, col + b)
            num += alpha[m] * (pi @ p.zeta)
            den += alpha[m] * pi.sum()
        assert abs(mass[r] - den) <= 1e-12 * max(abs(den), 1e-300) + 1e-18
        if den > 0:
            np.testing.assert_allclose(xi[r], num / den, rtol=1e-12, atol=1e-15)
        else:
            np.testing.assert_array_equal(xi[r], p.xi[r])
