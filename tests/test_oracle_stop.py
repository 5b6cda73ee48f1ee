"""Pins of the oracle's stopping tests (Sec. 5, stopping criteria) (CPU only).

* gamma = 0 on a line with a zero-diagonal cost whose off-diagonal gaps
  exceed rho * q_s: every plan becomes diag(q^(m)) after one iteration and
  stays there (up to rounding: the threshold q_s/R - q_s is subtracted back),
  so each test's values and the stopping iteration have closed forms;
* tol = -1 never stops and reproduces the plain run; tol = inf stops at the
  first check;
* the values of ||p^{k+1} - p^k|| match the p history of the plain run.
"""
import math

import numpy as np
import pytest

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def line_case(seed=0, R=7, M=3):
    # rho = 0.5: the smallest off-diagonal gap of w is 1/rho = 2 > q_s
    p = inputs.line_problem(seed, R=R, M=M, rho=0.5, gamma=0.0)
    cost, q = blocks(p)
    return p, cost, q


ROUND = 1e-15   # well above the rounding of q_s - (q_s/R - q_s) ~ 1e-17


def test_gamma_zero_line_dtheta_closed_form():
    p, cost, q = line_case()
    out = O.mam_until(cost, q, p.rho, 50, "dtheta", ROUND, 1, gamma=0.0)
    # theta^0 = q_s/R everywhere, theta^1 = diag(q): the largest change is
    # max_s max(q_s - q_s/R, q_s/R) = max_s q_s (1 - 1/R); theta^2 = theta^1
    first = max(float(qm.max()) * (1 - 1 / p.R) for qm in q)
    assert out["iters"] == 2 and out["converged"]
    assert out["values"][0] == pytest.approx(first, rel=1e-12)
    assert out["values"][1] <= 1e-16
    for th, qm in zip(out["theta"], q):
        np.testing.assert_allclose(th, np.diag(qm), rtol=0, atol=1e-16)


def test_gamma_zero_line_dp_closed_form():
    p, cost, q = line_case(1)
    out = O.mam_until(cost, q, p.rho, 50, "dp", ROUND, 1, gamma=0.0)
    a = np.array([1.0 / s for s in p.S])
    a /= a.sum()
    # p^0 = 1/R (unit masses), p^1 = sum_m a_m q^(m), p^2 = p^1
    p1 = sum(am * qm for am, qm in zip(a, q))
    assert out["iters"] == 2
    assert out["values"][0] == pytest.approx(float(np.linalg.norm(p1 - 1.0 / p.R)), rel=1e-12)
    assert out["values"][1] <= 1e-16


def test_gamma_zero_line_dist_closed_form():
    p, cost, q = line_case(2)
    a = np.array([1.0 / s for s in p.S])
    a /= a.sum()
    # pi_hat = diag(q^(m)) at every iteration: its row sums are q^(m)
    ph = sum(am * qm for am, qm in zip(a, q))
    dist = math.sqrt(sum(float(((ph - qm) ** 2).sum()) / s for qm, s in zip(q, p.S)))
    never = O.mam_until(cost, q, p.rho, 6, "dist", dist * (1 - 1e-9), 2, gamma=0.0)
    assert never["iters"] == 6 and not never["converged"]
    assert never["values"] == pytest.approx([dist] * 3, rel=1e-12)
    once = O.mam_until(cost, q, p.rho, 6, "dist", dist * (1 + 1e-9), 2, gamma=0.0)
    assert once["iters"] == 2 and once["converged"]


@pytest.mark.parametrize("every,expect", [(1, 2), (2, 2), (3, 3), (5, 5)])
def test_check_period(every, expect):
    p, cost, q = line_case(3)
    out = O.mam_until(cost, q, p.rho, 40, "dtheta", ROUND, every, gamma=0.0)
    assert out["iters"] == expect
    assert out["values"][-1] <= 1e-16 and len(out["values"]) == expect // every


@pytest.mark.parametrize("test", O.STOP_TESTS)
def test_never_and_immediate(test):
    p = inputs.tiny_problem(4, R=9, S=[5, 7, 6])
    cost, q = blocks(p)
    ref = O.mam(cost, q, p.rho, iters=11)
    never = O.mam_until(cost, q, p.rho, 11, test, -1.0, 3)
    assert never["iters"] == 11 and not never["converged"] and len(never["values"]) == 3
    np.testing.assert_array_equal(never["p_bar"], ref["p_bar"])
    for a_, b_ in zip(never["theta"], ref["theta"]):
        np.testing.assert_array_equal(a_, b_)
    first = O.mam_until(cost, q, p.rho, 11, test, math.inf, 4)
    assert first["iters"] == 4 and first["converged"]
    empty = O.mam_until(cost, q, p.rho, 0, test, math.inf, 1)
    assert empty["iters"] == 0 and empty["values"] == []


def test_dp_values_follow_p_history():
    p = inputs.tiny_problem(5, R=8, S=[6, 4])
    cost, q = blocks(p)
    ref = O.mam(cost, q, p.rho, iters=9, record=True)
    hist = ref["hist"]["p"]
    out = O.mam_until(cost, q, p.rho, 8, "dp", -1.0, 1)
    expect = [float(np.linalg.norm(hist[j] - hist[j - 1])) for j in range(1, 9)]
    assert out["values"] == pytest.approx(expect, rel=1e-12, abs=1e-300)


def test_dist_vanishes_at_balanced_convergence():
    # balanced DR: pi_hat^k approaches the balanced set (Sec. 5); the dist
    # test with a small tolerance eventually stops
    p = inputs.tiny_problem(6, R=6, S=[4, 5])
    cost, q = blocks(p)
    out = O.mam_until(cost, q, 5.0, 20000, "dist", 1e-9, 10)
    assert out["converged"] and out["values"][-1] <= 1e-9


def test_bad_arguments():
    p, cost, q = line_case()
    with pytest.raises(ValueError):
        O.mam_until(cost, q, 1.0, 5, "nope", 0.0, 1)
    with pytest.raises(ValueError):
        O.mam_until(cost, q, 1.0, 5, "dp", 0.0, 0)
