"""Pins of the oracle's support step (Prop. 4) and of the alternation (Alg. 2)
against facts fixed by the mathematics, not by the formula itself:

* a row whose mass sits on one point per measure moves to the alpha- and
  mass-weighted mean of those points (hand-computed values);
* the result minimises Psi(xi) = sum_m alpha_m sum_rs 1/2 ||xi_r - zeta_s||^2 pi_rs:
  the gradient, summed entry by entry in plain loops, vanishes, a general
  minimiser (scipy, from a random start) finds the same points, and every
  perturbation raises Psi;
* translating every measure's points translates the support; scaling alpha
  changes nothing; the points stay in the box of the measures' points;
* a row with no mass keeps its point;
* on line problems with gamma = 0 the plans are diag(q^(m)) after one
  iteration, so the alternation keeps a support equal to the shared points.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def rand_case(seed, R=7, S=(5, 4, 6), d=2):
    rng = np.random.default_rng(seed)
    pi = [rng.uniform(0, 1, size=(R, s)) * (rng.uniform(size=(R, s)) < 0.6) for s in S]
    zeta = [rng.normal(size=(s, d)) for s in S]
    alpha = rng.uniform(0.2, 1.0, size=len(S))
    xi_old = rng.normal(size=(R, d))
    return pi, zeta, alpha, xi_old


def psi(xi, pi, zeta, alpha):
    tot = 0.0
    for m in range(len(pi)):
        for r in range(pi[m].shape[0]):
            for s in range(pi[m].shape[1]):
                diff = xi[r] - zeta[m][s]
                tot += alpha[m] * 0.5 * float(diff @ diff) * pi[m][r, s]
    return tot


def test_single_point_rows_hand_values():
    # row 0: measure 0 puts 0.3 on (1, 0), measure 1 puts 0.1 on (0, 2);
    # alpha = (1, 2): xi_0 = (1*0.3*(1,0) + 2*0.1*(0,2)) / (0.3 + 0.2) = (0.6, 0.8)
    pi = [np.array([[0.3, 0.0], [0.0, 0.5]]), np.array([[0.0, 0.1], [0.4, 0.0]])]
    zeta = [np.array([[1.0, 0.0], [3.0, 3.0]]), np.array([[-1.0, 1.0], [0.0, 2.0]])]
    alpha = [1.0, 2.0]
    out = O.support_update(pi, zeta, alpha, np.zeros((2, 2)))
    np.testing.assert_allclose(out["xi"][0], [0.6, 0.8], rtol=0, atol=1e-15)
    # row 1: 1*0.5*(3,3) + 2*0.4*(-1,1) over 0.5 + 0.8 = (0.7, 2.3)/1.3
    np.testing.assert_allclose(out["xi"][1], [0.7 / 1.3, 2.3 / 1.3], rtol=1e-15)
    np.testing.assert_allclose(out["mass"], [0.5, 1.3], rtol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_of_psi_vanishes(seed):
    pi, zeta, alpha, xi_old = rand_case(seed)
    xi = O.support_update(pi, zeta, alpha, xi_old)["xi"]
    for r in range(xi.shape[0]):
        g = np.zeros(xi.shape[1])
        scale = 0.0
        for m in range(len(pi)):
            for s in range(pi[m].shape[1]):
                g += alpha[m] * (xi[r] - zeta[m][s]) * pi[m][r, s]
                scale += alpha[m] * pi[m][r, s] * (np.abs(zeta[m][s]).max() + np.abs(xi[r]).max())
        assert np.abs(g).max() <= 1e-13 * max(scale, 1e-300)


def test_general_minimiser_agrees():
    pi, zeta, alpha, xi_old = rand_case(3, R=4, S=(3, 5), d=2)
    xi = O.support_update(pi, zeta, alpha, xi_old)["xi"]
    x0 = np.random.default_rng(9).normal(size=xi.size)
    res = minimize(lambda v: psi(v.reshape(xi.shape), pi, zeta, alpha), x0, method="BFGS",
                   options={"gtol": 1e-12})
    np.testing.assert_allclose(res.x.reshape(xi.shape), xi, rtol=0, atol=1e-6)
    base = psi(xi, pi, zeta, alpha)
    rng = np.random.default_rng(4)
    for _ in range(20):
        assert psi(xi + 1e-3 * rng.normal(size=xi.shape), pi, zeta, alpha) > base


def test_translation_scaling_and_box():
    pi, zeta, alpha, xi_old = rand_case(5, R=9, S=(6, 3, 7, 2), d=3)
    xi = O.support_update(pi, zeta, alpha, xi_old)["xi"]
    v = np.array([0.25, -3.0, 7.5])
    moved = O.support_update(pi, [z + v for z in zeta], alpha, xi_old)["xi"]
    np.testing.assert_allclose(moved, xi + v, rtol=0, atol=1e-13)
    scaled = O.support_update(pi, zeta, [5.0 * a for a in alpha], xi_old)["xi"]
    np.testing.assert_allclose(scaled, xi, rtol=1e-14, atol=1e-15)
    lo = np.min([z.min(axis=0) for z in zeta], axis=0)
    hi = np.max([z.max(axis=0) for z in zeta], axis=0)
    assert np.all(xi >= lo - 1e-14) and np.all(xi <= hi + 1e-14)


def test_rows_without_mass_keep_their_point():
    pi, zeta, alpha, xi_old = rand_case(6)
    for P in pi:
        P[2] = 0.0
    out = O.support_update(pi, zeta, alpha, xi_old)
    assert out["mass"][2] == 0.0
    np.testing.assert_array_equal(out["xi"][2], xi_old[2])


def test_alternation_keeps_shared_points_on_line_problems():
    # M measures on the barycenter's own points 0..R-1 of a line; with gamma = 0
    # one iteration gives diag(q^(m)), so every round moves xi_r to r exactly
    p = inputs.line_problem(1, R=6, M=3, gamma=0.0)
    x = np.arange(p.R, dtype=np.float64)[:, None]
    zeta = [x.copy() for _ in range(p.M)]
    q = [p.q_block(m) for m in range(p.M)]
    out = O.free_support_alternation(x + 0.0, zeta, q, [1.0 / p.M] * p.M, rho=0.5, gamma=0.0,
                                     outer=3, inner=2)
    for xi in out["xi"]:
        np.testing.assert_allclose(xi, x, rtol=0, atol=1e-12)


def test_alternation_composes_mam_and_support_step():
    p = inputs.tiny_problem(7, R=12, S=[9, 11], rho=2.0)
    rng = np.random.default_rng(2)
    xi0 = rng.uniform(0, 1, size=(p.R, 2))
    zeta = [rng.uniform(0, 1, size=(s, 2)) for s in p.S]
    q = [p.q_block(m) for m in range(p.M)]
    alpha = [0.3, 0.7]
    out = O.free_support_alternation(xi0, zeta, q, alpha, rho=2.0, outer=2, inner=3)
    c0 = [alpha[m] * 0.5 * O.sq_euclid_cost(xi0, zeta[m]) for m in range(2)]
    r0 = O.mam(c0, q, 2.0, iters=3)
    xi1 = O.support_update(r0["pi_hat"], zeta, alpha, xi0)["xi"]
    np.testing.assert_array_equal(out["xi"][0], xi1)
    c1 = [alpha[m] * 0.5 * O.sq_euclid_cost(xi1, zeta[m]) for m in range(2)]
    r1 = O.mam(c1, q, 2.0, iters=3, theta0=r0["theta"])
    np.testing.assert_array_equal(out["xi"][1], O.support_update(r1["pi_hat"], zeta, alpha, xi1)["xi"])
    # the support step never raises the transport objective of the plans it is given
    assert psi(xi1, r0["pi_hat"], zeta, alpha) <= psi(xi0, r0["pi_hat"], zeta, alpha)
