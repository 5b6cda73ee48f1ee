"""Pins of the full unbalanced extension in the oracle (CPU only): the
projection onto {u >= 0, sum u <= tau} against its optimality conditions and
a brute-force minimiser, and runs to convergence against the relaxed problem
minimised directly by SLSQP."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import lp
from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def brute_subsimplex(w, tau):
    x0 = np.full(w.size, tau / (2 * w.size))
    res = minimize(lambda x: 0.5 * ((x - w) ** 2).sum(), x0, jac=lambda x: x - w, method="SLSQP",
                   bounds=[(0, None)] * w.size,
                   constraints=[{"type": "ineq", "fun": lambda x: tau - x.sum(), "jac": lambda x: -np.ones_like(x)}],
                   options={"ftol": 1e-15, "maxiter": 500})
    return res.x


@pytest.mark.parametrize("seed", range(20))
def test_subsimplex_projection(seed):
    rng = np.random.default_rng([41, seed])
    R = int(rng.integers(1, 7))
    w = rng.normal(0, 1, R) * rng.choice([0.01, 0.3, 2.0])
    tau = float(rng.choice([0.0, 0.05, 0.5, 3.0]))
    x = O.proj_subsimplex(w[:, None], [tau])[:, 0]
    # optimality: x = max(w - mu, 0) with mu >= 0, sum x <= tau, mu (tau - sum x) = 0
    assert np.all(x >= 0) and x.sum() <= tau + 1e-12
    if x.sum() < tau - 1e-12:
        np.testing.assert_allclose(x, np.maximum(w, 0), atol=1e-15)
    elif tau > 0:
        mu = np.max(w - x)
        assert mu >= -1e-12
        np.testing.assert_allclose(x, np.maximum(w - mu, 0), atol=1e-12)
    if tau > 0:
        np.testing.assert_allclose(x, brute_subsimplex(w, tau), atol=1e-6)
    else:
        assert np.all(x == 0)


def test_subsimplex_special_cases():
    w = np.array([[-1.0, 0.2], [-0.5, 0.1], [-2.0, 0.05]])
    x = O.proj_subsimplex(w, [1.0, 1.0])
    assert np.all(x[:, 0] == 0)                                 # nothing positive
    np.testing.assert_array_equal(x[:, 1], [0.2, 0.1, 0.05])    # fits: clamped vector kept
    x = O.proj_subsimplex(np.array([[3.0], [1.0]]), [1.0])
    np.testing.assert_allclose(x[:, 0], [1.0, 0.0])             # w_1 - w_2 >= tau: all on the first


@pytest.mark.parametrize("seed,gamma,eta", [(21, 0.2, 0.1), (23, 0.2, 0.1), (21, 0.2, 0.2)])
def test_relaxed_run_reaches_the_relaxed_optimum(seed, gamma, eta):
    p = inputs.tiny_problem(seed, R=4, S=[3, 3], masses=[0.7, 1.3], gamma=gamma)
    cost, q = blocks(p)
    d = [c - eta for c in cost]  # the shifted distances of the extension
    f_ref, _ = lp.uwb_slsqp(d, q, gamma, relaxed=True, iters=3000)
    r = O.mam(d, q, 1.0, gamma=gamma, iters=20000, relaxed=True)
    f = lp.uwb_objective(d, r["pi_hat"], gamma)
    assert f <= f_ref + 1e-8
    assert abs(f - f_ref) < 1e-6
    slack = min(float((ph.sum(axis=0) - qm).min()) for ph, qm in zip(r["pi_hat"], q))
    for ph, qm in zip(r["pi_hat"], q):
        assert np.all(ph >= 0) and np.all(ph.sum(axis=0) <= qm + 1e-12)
    if eta < 0.15:
        assert slack < -1e-3  # some mass stays untransported: the relaxation is active


def test_relaxed_with_no_profitable_transport_is_zero():
    # eta below every cost: leaving all mass in place is optimal
    p = inputs.tiny_problem(22, R=4, S=[3, 3], masses=[0.7, 1.3], gamma=0.2)
    cost, q = blocks(p)
    eta = 0.5 * min(float(c.min()) for c in cost)
    r = O.mam([c - eta for c in cost], q, 1.0, gamma=0.2, iters=5000, relaxed=True)
    assert max(float(np.abs(ph).max()) for ph in r["pi_hat"]) < 1e-9


def test_relaxed_equals_plain_when_every_column_overflows():
    # with large w (no cost shift, positive entries) every clamped column
    # carries more than q_s, so both projections agree
    p = inputs.tiny_problem(22, R=5, S=[4, 3])
    cost, q = blocks(p)
    shifted = [c - 10.0 for c in cost]
    a = O.mam(shifted, q, 1.0, iters=30)
    b = O.mam(shifted, q, 1.0, iters=30, relaxed=True)
    np.testing.assert_allclose(a["p_bar"], b["p_bar"], rtol=0, atol=1e-14)
