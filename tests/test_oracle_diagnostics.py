"""Pins of the oracle's per-iteration figures and of its parallel driver.

* ``diagnostics``: W_hat = sum_m <c^(m), pi_hat^(m)> (the objective reported
  in Sec. 6.3), dist_L(pi_hat), the measure residual max_{m,s} |sum_r
  pi_hat_rs - q_s| and ||theta^{k+1} - theta^k||_inf (the stopping tests of
  Sec. 5), on hand-built plans whose values are exact in binary, so every
  figure is known in closed form.
* ``dist_L_marginals``: Prop. 2 puts the distance to L in terms of the
  marginals alone; checked against the distance to the projection.
* ``mam_parallel`` (the paper's scheme of one process per group of
  measures): equal bit for bit to the one-process oracle.
"""
import functools
import math

import numpy as np
import pytest

from oracle import mam_oracle as O
from oracle.mam_parallel import mam_parallel
from paper_2309_05315_amd import inputs


def hand_case():
    # two measures, R = 3; plans with binary-exact entries
    c = [np.array([[1.0, 2.0], [3.0, 4.0], [0.5, 0.0]]),
         np.array([[2.0], [0.0], [8.0]])]
    q = [np.array([0.5, 0.25]), np.array([0.75])]
    ph = [np.array([[0.5, 0.0], [0.0, 0.125], [0.0, 0.0]]),   # column sums 0.5, 0.125
          np.array([[0.25], [0.5], [0.0]])]                   # column sum 0.75
    th_old = [np.array([[0.5, 0.0], [0.0, 0.25], [0.0, 0.0]]),
              np.array([[0.0], [0.5], [0.25]])]
    th_new = [np.array([[0.5, 0.0625], [0.0, 0.25], [0.0, 0.0]]),
              np.array([[0.25], [0.5], [-0.125]])]
    return c, q, ph, th_new, th_old


def test_diagnostics_hand_values():
    c, q, ph, th_new, th_old = hand_case()
    d = O.diagnostics(c, q, ph, th_new, th_old)
    # <c1, ph1> = 1*0.5 + 4*0.125 = 1; <c2, ph2> = 2*0.25 + 0*0.5 = 0.5
    assert d["W_hat"] == 1.5
    # column sums 0.5, 0.125, 0.75 against q = 0.5, 0.25, 0.75
    assert d["meas_resid"] == 0.125
    # the largest change is theta2[2] from 0.25 to -0.125 (a sign change)
    assert d["dtheta_inf"] == 0.375
    # dist_L by hand: S = (2, 1), a = (1/3, 2/3); marginals of pi_hat
    pm = np.array([[0.5, 0.125, 0.0], [0.25, 0.5, 0.0]])
    p = pm[0] / 3 + 2 * pm[1] / 3
    want = math.sqrt(((p - pm[0]) ** 2).sum() / 2 + ((p - pm[1]) ** 2).sum() / 1)
    assert d["dist_L"] == pytest.approx(want, rel=1e-15)


def test_diagnostics_each_figure_moves_with_its_own_entry():
    """A planted change in one entry moves only the figure that reads it."""
    c, q, ph, th_new, th_old = hand_case()
    base = O.diagnostics(c, q, ph, th_new, th_old)
    th2 = [t.copy() for t in th_new]
    th2[0][1, 0] = 0.5          # |0.5 - 0| = 0.5 > 0.375
    d = O.diagnostics(c, q, ph, th2, th_old)
    assert d["dtheta_inf"] == 0.5 and d["W_hat"] == base["W_hat"] and d["meas_resid"] == base["meas_resid"]
    q2 = [q[0].copy(), q[1] - 0.25]  # column of measure 2 now over by 0.25
    d = O.diagnostics(c, q2, ph, th_new, th_old)
    assert d["meas_resid"] == 0.25 and d["dtheta_inf"] == base["dtheta_inf"]
    ph2 = [ph[0].copy(), ph[1].copy()]
    ph2[1][2, 0] = 0.125        # cost 8 -> W_hat grows by 1
    d = O.diagnostics(c, q, ph2, th_new, th_old)
    assert d["W_hat"] == 2.5


def test_dist_L_from_marginals_is_the_distance_to_the_projection():
    rng = np.random.default_rng(4)
    th = [rng.normal(size=(5, s)) for s in (3, 7, 4)]
    pi, _, _ = O.proj_L(th)
    direct = math.sqrt(sum(float(((a - b) ** 2).sum()) for a, b in zip(th, pi)))
    assert O.dist_L_marginals(O.marginals(th), [3, 7, 4]) == pytest.approx(direct, rel=1e-12)
    assert O.dist_L(th) == O.dist_L_marginals(O.marginals(th), [3, 7, 4])


@pytest.mark.parametrize("gamma,workers", [(math.inf, 2), (0.05, 3), (0.05, 8)])
def test_parallel_scheme_equals_one_process_bitwise(gamma, workers):
    masses = None if math.isinf(gamma) else [0.7, 1.0, 1.3, 0.9, 1.1]
    build = functools.partial(inputs.tiny_problem, 5, R=60, S=[7, 12, 9, 4, 10], masses=masses, gamma=gamma)
    p = build()
    cost = [p.cost_block(m) for m in range(p.M)]
    q = [p.q_block(m) for m in range(p.M)]
    K = 7
    prev = O.mam(cost, q, p.rho, p.gamma, K - 1)
    ora = O.mam(cost, q, p.rho, p.gamma, K)
    od = O.diagnostics(cost, q, ora["pi_hat"], ora["theta"], prev["theta"])
    r = mam_parallel(build, K, workers)
    assert np.array_equal(r["p_bar"], ora["p_bar"])
    assert np.array_equal(r["pm"], ora["pm"])
    assert r["t"] == ora["t"]
    for k in ("W_hat", "dist_L", "meas_resid", "dtheta_inf"):
        assert r[k] == od[k], k
    if not math.isinf(gamma):
        assert r["t"] < 1.0
