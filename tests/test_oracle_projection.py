"""Pins of the oracle's column projection and of Prop. 2 (CPU only).

The oracle's sort-based projection is checked against things other than its
own formula: hand-solved cases, the KKT conditions of the projection, a
bisection on the threshold (a different algorithm), SLSQP on tiny columns,
and special cases with known answers.  Prop. 2 is checked against a
least-squares projection onto the constraint subspace L written out densely.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

from oracle import mam_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def kkt_residual(w, tau, x):
    """Largest violation of the optimality conditions of min ||x-w||^2 on Delta(tau):
    x >= 0, sum x = tau, and a common lambda with w - x = lambda on x > 0 and
    w <= lambda on x = 0."""
    viol = max(0.0, -x.min())
    viol = max(viol, abs(x.sum() - tau))
    act = x > 0
    if tau == 0:
        return max(viol, np.abs(x).max())
    lam = np.mean((w - x)[act])
    viol = max(viol, np.abs((w - x)[act] - lam).max())
    if (~act).any():
        viol = max(viol, max(0.0, (w[~act] - lam).max()))
    return viol


def proj_bisect(w, tau, iters=200):
    """Threshold by bisection on the monotone map lambda -> sum max(w - lambda, 0)."""
    if tau == 0:
        return np.zeros_like(w)
    lo, hi = w.max() - tau, w.max()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.maximum(w - mid, 0).sum() > tau:
            lo = mid
        else:
            hi = mid
    return np.maximum(w - 0.5 * (lo + hi), 0)


def test_golden_hand_cases():
    with open(os.path.join(GOLD, "simplex_projection.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        x, _ = O.proj_simplex_sort(np.array(c["w"]), c["tau"])
        np.testing.assert_allclose(x, c["expect"], rtol=0, atol=1e-15, err_msg=c["derivation"])


@pytest.mark.parametrize("seed", range(6))
def test_kkt_random(seed):
    rng = np.random.default_rng(seed)
    R, n = [1, 2, 7, 64, 300, 1025][seed], 40
    w = rng.normal(size=(R, n)) * rng.uniform(0.01, 10)
    tau = rng.uniform(0, 3, size=n)
    tau[::7] = 0.0
    x, lam = O.proj_simplex_sort(w, tau)
    for s in range(n):
        assert kkt_residual(w[:, s], tau[s], x[:, s]) < 1e-12 * max(1.0, np.abs(w).max())
        if tau[s] > 0:
            np.testing.assert_allclose(x[:, s], np.maximum(w[:, s] - lam[s], 0), atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_against_bisection(seed):
    rng = np.random.default_rng(100 + seed)
    R = [5, 33, 256, 4096][seed]
    w = rng.normal(size=(R, 8)) - rng.uniform(0, 1, size=(R, 1))
    tau = rng.uniform(1e-6, 2, size=8)
    x, _ = O.proj_simplex_sort(w, tau)
    for s in range(8):
        np.testing.assert_allclose(x[:, s], proj_bisect(w[:, s], tau[s]), atol=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_against_slsqp(seed):
    rng = np.random.default_rng(200 + seed)
    R = 2 + seed
    w = rng.normal(size=R)
    tau = rng.uniform(0.1, 2)
    res = minimize(lambda x: ((x - w) ** 2).sum(), np.full(R, tau / R),
                   jac=lambda x: 2 * (x - w), method="SLSQP",
                   bounds=[(0, None)] * R,
                   constraints=[{"type": "eq", "fun": lambda x: x.sum() - tau,
                                 "jac": lambda x: np.ones(R)}],
                   options={"ftol": 1e-15, "maxiter": 500})
    x, _ = O.proj_simplex_sort(w, tau)
    np.testing.assert_allclose(x, res.x, atol=1e-7)


def test_special_cases():
    # all-equal entries share tau equally
    x, _ = O.proj_simplex_sort(np.full(10, 3.25), 0.5)
    np.testing.assert_allclose(x, np.full(10, 0.05), atol=1e-16)
    # a gap of at least tau puts all mass on the top entry
    w = np.array([0.0, 1.5, -0.2, 0.4])
    x, _ = O.proj_simplex_sort(w, 1.1)
    np.testing.assert_allclose(x, [0, 1.1, 0, 0], atol=1e-15)
    # R = 1 and tau = 0
    assert abs(O.proj_simplex_sort(np.array([-9.0]), 0.3)[0][0] - 0.3) < 1e-14
    assert not O.proj_simplex_sort(np.array([1.0, 2.0]), 0.0)[0].any()
    # translation invariance: Proj(w + c) = Proj(w)
    w = np.random.default_rng(3).normal(size=50)
    np.testing.assert_allclose(O.proj_simplex_sort(w + 123.0, 0.7)[0],
                               O.proj_simplex_sort(w, 0.7)[0], atol=1e-12)


def test_tiny_tau_gives_zero_column_not_nan():
    # tau far below the rounding resolution of w: no division by zero
    w = np.array([1.0, 0.5, 0.25])
    x, lam = O.proj_simplex_sort(w, 1e-87)
    assert np.isfinite(x).all() and np.isfinite(lam)
    assert abs(x.sum() - 1e-87) <= 1e-87


# ---------------------------------------------------------------------------
# Prop. 2: Proj_L
# ---------------------------------------------------------------------------
def _proj_L_lstsq(theta):
    """Orthogonal projection onto L by least squares on its dense constraint
    matrix: rows encode p^(m)_r - p^(m+1)_r = 0 for every r and m < M."""
    R = theta[0].shape[0]
    S = [t.shape[1] for t in theta]
    n = R * sum(S)
    offs = np.concatenate([[0], np.cumsum([R * s for s in S])])
    rows = []
    for m in range(len(S) - 1):
        for r in range(R):
            row = np.zeros(n)
            row[offs[m] + r * S[m]: offs[m] + (r + 1) * S[m]] = 1.0
            row[offs[m + 1] + r * S[m + 1]: offs[m + 1] + (r + 1) * S[m + 1]] = -1.0
            rows.append(row)
    A = np.array(rows)
    x = np.concatenate([t.ravel() for t in theta])
    y, *_ = np.linalg.lstsq(A @ A.T, A @ x, rcond=None)
    xp = x - A.T @ y
    return [xp[offs[m]:offs[m + 1]].reshape(R, S[m]) for m in range(len(S))]


def test_proj_L_golden():
    with open(os.path.join(GOLD, "proj_L.json")) as f:
        g = json.load(f)
    theta = [np.array(t) for t in g["theta"]]
    pi, p, _ = O.proj_L(theta)
    np.testing.assert_allclose(O.averaging_weights([1, 2]), g["a"], atol=1e-16)
    np.testing.assert_allclose(p, g["p"], atol=1e-15)
    for a, b in zip(pi, g["pi"]):
        np.testing.assert_allclose(a, b, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_proj_L_vs_lstsq(seed):
    rng = np.random.default_rng(300 + seed)
    R = [2, 3, 5, 6][seed]
    S = [[1, 3], [2, 4, 3], [5, 1, 2, 7], [3, 3, 3]][seed]
    theta = [rng.normal(size=(R, s)) for s in S]
    pi, _, _ = O.proj_L(theta)
    ref = _proj_L_lstsq(theta)
    for a, b in zip(pi, ref):
        np.testing.assert_allclose(a, b, atol=1e-12)
    # pi in L: equal row sums; theta - pi orthogonal to L
    rs = [x.sum(axis=1) for x in pi]
    for r in rs[1:]:
        np.testing.assert_allclose(r, rs[0], atol=1e-12)
    # dist_L reduction to R-vectors equals the Frobenius distance
    dF = math.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(theta, ref)))
    assert abs(O.dist_L(theta) - dF) < 1e-12


@pytest.mark.parametrize("gamma", [0.0, 0.05, 0.3, 5.0])
def test_unbalanced_prox_vs_line_search(gamma):
    """eq. (Unbalanced-prox) against a direct scalar minimisation of
    gamma*dist_L(pi) + rho/2 ||pi - theta||^2 along theta -> Proj_L(theta)
    (the minimiser lies on that segment), and against random perturbations."""
    rng = np.random.default_rng(7)
    rho = 2.0
    theta = [rng.normal(size=(4, s)) for s in (2, 3, 5)]
    P = _proj_L_lstsq(theta)
    D = [pp - t for pp, t in zip(P, theta)]

    def obj_pi(pi):
        return gamma * O.dist_L(pi) + 0.5 * rho * sum(((a - b) ** 2).sum() for a, b in zip(pi, theta))

    res = minimize_scalar(lambda s: obj_pi([t + s * d for t, d in zip(theta, D)]),
                          bounds=(0, 1), method="bounded", options={"xatol": 1e-13})
    ref = [t + res.x * d for t, d in zip(theta, D)]
    got = O.unbalanced_prox(theta, rho, gamma)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, atol=1e-8)
    f0 = obj_pi(got)
    for _ in range(50):
        pert = [g + 1e-4 * rng.normal(size=g.shape) for g in got]
        assert obj_pi(pert) >= f0 - 1e-12
