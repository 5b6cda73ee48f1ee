"""Pins of the oracle's Alg. 1 (CPU only).

* one fused Alg. 1 step equals the three-line DR scheme (eq. (DR)) evaluated
  with independently computed proximal maps (least-squares Proj_L, threshold
  bisection for the simplex columns);
* runs to convergence reach the optimum of the LP (HugeLP) solved by HiGHS,
  and, unbalanced, the optimum of (UWB) found by SLSQP;
* special cases with a unique known barycenter;
* the mass and column-sum invariants of every iteration;
* the DR map is nonexpansive.
"""
import math

import numpy as np
import pytest

from oracle import lp
from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def _bisect_cols(w, tau):
    out = np.zeros_like(w)
    for s in range(w.shape[1]):
        if tau[s] == 0:
            continue
        lo, hi = w[:, s].max() - tau[s], w[:, s].max()
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if np.maximum(w[:, s] - mid, 0).sum() > tau[s]:
                lo = mid
            else:
                hi = mid
        out[:, s] = np.maximum(w[:, s] - 0.5 * (lo + hi), 0)
    return out


def _lstsq_PL(theta):
    R = theta[0].shape[0]
    S = [t.shape[1] for t in theta]
    n = R * sum(S)
    offs = np.concatenate([[0], np.cumsum([R * s for s in S])])
    A = []
    for m in range(len(S) - 1):
        for r in range(R):
            row = np.zeros(n)
            row[offs[m] + r * S[m]: offs[m] + (r + 1) * S[m]] = 1
            row[offs[m + 1] + r * S[m + 1]: offs[m + 1] + (r + 1) * S[m + 1]] = -1
            A.append(row)
    A = np.array(A)
    x = np.concatenate([t.ravel() for t in theta])
    y, *_ = np.linalg.lstsq(A @ A.T, A @ x, rcond=None)
    xp = x - A.T @ y
    return [xp[offs[m]:offs[m + 1]].reshape(R, S[m]) for m in range(len(S))]


def dr_textbook_step(theta, cost, q, rho, gamma):
    """eq. (DR): pi = prox_{g/rho}(theta); pi_hat = prox_{f/rho}(2 pi - theta);
    theta' = theta + pi_hat - pi, with g = indicator of L (balanced) or
    gamma*dist_L, f = <c, .> + indicator of Pi; each prox computed from its
    definition (lstsq projection; the prox of gamma*dist_L moves theta toward
    its projection by min(1, gamma/(rho*dist)); the prox of f shifts by -c/rho
    and projects every column by bisection)."""
    P = _lstsq_PL(theta)
    dist = math.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(P, theta)))
    step = 1.0 if (math.isinf(gamma) or rho * dist <= gamma) else gamma / (rho * dist)
    pi = [t + step * (pp - t) for t, pp in zip(theta, P)]
    pi_hat = [_bisect_cols(2 * p_ - t - c / rho, qm) for p_, t, c, qm in zip(pi, theta, cost, q)]
    return [t + ph - p_ for t, ph, p_ in zip(theta, pi_hat, pi)]


@pytest.mark.parametrize("gamma", [math.inf, 0.02, 0.3])
@pytest.mark.parametrize("seed", range(3))
def test_fused_step_equals_textbook_dr(seed, gamma):
    masses = None if math.isinf(gamma) else [0.6, 1.0, 1.4]
    p = inputs.tiny_problem(seed, R=5, S=[3, 4, 2], masses=masses, gamma=gamma)
    cost, q = blocks(p)
    rng = np.random.default_rng(seed)
    theta = [rng.normal(scale=0.2, size=(5, s)) for s in p.S]
    for rho in (0.5, 3.0):
        ref = dr_textbook_step(theta, cost, q, rho, gamma)
        got, pm_new, _ = O.mam_step(theta, O.marginals(theta), cost, q, rho, gamma)
        for a, b in zip(got, ref):
            np.testing.assert_allclose(a, b, atol=1e-11)
        np.testing.assert_allclose(pm_new, O.marginals(ref), atol=1e-11)


@pytest.mark.parametrize("seed", range(4))
def test_converges_to_lp_optimum(seed):
    p = inputs.tiny_problem(seed, R=[6, 9, 8, 12][seed], S=[[4, 5], [5, 7, 6], [3, 8, 2, 5], [6, 6]][seed],
                            zero_frac=0.0 if seed < 3 else 0.0, shared=(seed == 3))
    cost, q = blocks(p)
    f_lp, _, _ = lp.wb_lp(cost, q)
    r = O.mam(cost, q, 1.0, iters=4000)
    d = O.diagnostics(cost, q, r["pi_hat"], r["theta"], r["theta"])
    assert abs(d["W_hat"] - f_lp) <= 1e-6 * max(1.0, abs(f_lp))
    assert d["dist_L"] < 1e-6
    assert r["p_bar"].min() > -1e-8
    assert abs(r["p_bar"].sum() - 1.0) < 1e-10


def test_non_square_cost_orientation():
    """c^(m) is R x S^m: a transposed cost would not even have the right shape
    here, and the LP optimum pins which index is the barycenter side."""
    xi = np.array([[0.0], [0.5], [1.0]])             # barycenter support (R=3)
    z1 = np.array([[0.0], [0.1]])                     # measure 1 (S=2)
    z2 = np.array([[0.9], [1.0], [0.8], [0.2]])      # measure 2 (S=4)
    cost = [O.sq_euclid_cost(xi, z1), O.sq_euclid_cost(xi, z2)]
    q = [np.array([0.5, 0.5]), np.array([0.25, 0.25, 0.25, 0.25])]
    f_lp, _, _ = lp.wb_lp(cost, q)
    r = O.mam(cost, q, 1.0, iters=5000)
    d = O.diagnostics(cost, q, r["pi_hat"], r["theta"], r["theta"])
    assert abs(d["W_hat"] - f_lp) < 1e-7


def test_delta_barycenter_on_a_line():
    """nu1 = delta at x0 = 0, nu2 = delta at x4 = 1 on 5 equispaced points:
    the unique barycenter is the delta at the midpoint x2."""
    x = np.linspace(0, 1, 5)[:, None]
    cost = [O.sq_euclid_cost(x, x[[0]]), O.sq_euclid_cost(x, x[[4]])]
    r = O.mam(cost, [np.ones(1), np.ones(1)], 1.0, iters=500)
    np.testing.assert_allclose(r["p_bar"], [0, 0, 1, 0, 0], atol=1e-12)


def test_identical_measures_reproduce_them():
    """Identical measures on the barycenter grid with zero diagonal cost:
    the barycenter is the measure itself (the diagonal plan costs 0)."""
    p = inputs.balanced_plain(K=4, M=3)
    cost, _ = blocks(p)
    q0 = p.q_block(0)
    r = O.mam(cost, [q0, q0, q0], 1.0, iters=3000)
    np.testing.assert_allclose(r["p_bar"], q0, atol=1e-12)


def test_gamma_zero_decouples_measures():
    """gamma = 0 gives t = 0 while the marginals differ, so every plan follows
    theta' = Proj_Pi(theta - c/rho) alone and settles on the zero-cost
    diagonal: the barycenter is sum_m a_m q^(m)."""
    p = inputs.balanced_plain(K=4, M=3)
    cost, q = blocks(p)
    q = [qm * (m + 1) for m, qm in enumerate(q)]
    r = O.mam(cost, q, 1.0, gamma=0.0, iters=200, record=True)
    a = O.averaging_weights(p.S)
    np.testing.assert_allclose(r["p_bar"], sum(a[m] * q[m] for m in range(3)), atol=1e-14)
    assert max(r["hist"]["t"]) == 0.0


def test_large_finite_gamma_is_bitwise_balanced():
    p = inputs.balanced_plain(K=4, M=3)
    cost, q = blocks(p)
    r0 = O.mam(cost, q, 1.0, gamma=math.inf, iters=50, record=True)
    bound = 1.0 * max(r0["hist"]["d"])
    r1 = O.mam(cost, q, 1.0, gamma=bound * 1.0000001, iters=50)
    assert np.array_equal(r0["p_bar"], r1["p_bar"])
    for a, b in zip(r0["theta"], r1["theta"]):
        assert np.array_equal(a, b)


def test_exact_penalty_recovers_balanced_objective():
    """Prop. prop_gamma: on probability measures gamma > ||vec(c)|| gives a WB."""
    p = inputs.tiny_problem(11, R=6, S=[4, 5])
    cost, q = blocks(p)
    gamma = 1.01 * math.sqrt(sum((c ** 2).sum() for c in cost))
    f_lp, _, _ = lp.wb_lp(cost, q)
    r = O.mam(cost, q, 1.0, gamma=gamma, iters=4000)
    d = O.diagnostics(cost, q, r["pi_hat"], r["theta"], r["theta"])
    assert abs(d["W_hat"] - f_lp) < 1e-7


@pytest.mark.parametrize("gamma", [0.02, 0.05, 0.2])
def test_unbalanced_reaches_uwb_optimum(gamma):
    p = inputs.tiny_problem(3, R=4, S=[3, 3], masses=[0.7, 1.3], gamma=gamma)
    cost, q = blocks(p)
    f_ref, _ = lp.uwb_slsqp(cost, q, gamma)
    r = O.mam(cost, q, 1.0, gamma=gamma, iters=20000)
    f = lp.uwb_objective(cost, r["pi_hat"], gamma)
    assert f <= f_ref + 1e-9
    assert abs(f - f_ref) < 1e-7
    assert r["t"] < 1.0          # masses differ: the damping is active at the fixed point


@pytest.mark.parametrize("gamma", [math.inf, 0.05])
def test_per_iteration_invariants(gamma):
    """Column sums of pi_hat equal q_s, and the mass of every marginal moves by
    sum_r p^(m),k+1 = sum q^(m) - t^k (sum p^k - sum p^(m),k)."""
    masses = None if math.isinf(gamma) else [0.5, 1.0, 1.5]
    p = inputs.tiny_problem(5, R=7, S=[4, 6, 5], masses=masses, zero_frac=0.2)
    cost, q = blocks(p)
    theta = [np.repeat((qm / 7)[None, :], 7, axis=0) for qm in q]
    pm = O.marginals(theta)
    for _ in range(30):
        theta, pm_new, info = O.mam_step(theta, pm, cost, q, 1.0, gamma)
        for ph, qm in zip(info["pi_hat"], q):
            np.testing.assert_allclose(ph.sum(axis=0), qm, atol=1e-15)
            assert ph.min() >= 0
        for m in range(3):
            expect = q[m].sum() - info["t"] * (info["p"].sum() - pm[m].sum())
            assert abs(pm_new[m].sum() - expect) < 1e-14
        pm = pm_new


@pytest.mark.parametrize("gamma", [math.inf, 0.1])
def test_dr_map_is_nonexpansive(gamma):
    p = inputs.tiny_problem(9, R=6, S=[5, 3, 4], masses=None if math.isinf(gamma) else [0.8, 1.0, 1.2])
    cost, q = blocks(p)
    rng = np.random.default_rng(1)
    for _ in range(20):
        A = [rng.normal(scale=0.3, size=(6, s)) for s in p.S]
        B = [a + rng.normal(scale=0.05, size=a.shape) for a in A]
        TA, _, _ = O.mam_step(A, O.marginals(A), cost, q, 1.3, gamma)
        TB, _, _ = O.mam_step(B, O.marginals(B), cost, q, 1.3, gamma)
        nA = math.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(TA, TB)))
        n0 = math.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(A, B)))
        assert nA <= n0 * (1 + 1e-12)


def test_init_and_return_readings():
    """theta^0 = q/R gives p^(m) = (sum q^(m))/R; zero iterations return the
    averaged marginal of theta^0 (the barycenter is sum_m a_m p^(m) of the
    final theta)."""
    p = inputs.tiny_problem(2, R=5, S=[3, 4])
    cost, q = blocks(p)
    r = O.mam(cost, q, 1.0, iters=0)
    np.testing.assert_allclose(r["p_bar"], np.full(5, 0.2), atol=1e-16)
    r1 = O.mam(cost, q, 1.0, iters=3)
    pi, p_proj, _ = O.proj_L(r1["theta"])
    np.testing.assert_allclose(r1["p_bar"], p_proj, atol=1e-16)


def test_sampled_columns_match_full_step():
    p = inputs.tiny_problem(4, R=9, S=[5, 7, 3], masses=[0.9, 1.0, 1.1])
    cost, q = blocks(p)
    rng = np.random.default_rng(0)
    theta = [rng.normal(scale=0.1, size=(9, s)) for s in p.S]
    pm = O.marginals(theta)
    full, _, _ = O.mam_step(theta, pm, cost, q, 1.7, 0.05)
    picks = [(0, 1), (1, 6), (2, 0), (1, 2)]
    cols = np.stack([theta[m][:, s] for m, s in picks], axis=1)
    ccols = np.stack([cost[m][:, s] for m, s in picks], axis=1)
    qcols = np.array([q[m][s] for m, s in picks])
    got, _, _ = O.mam_step_columns(cols, [m for m, _ in picks], pm, ccols, qcols, p.S, 1.7, 0.05)
    for k, (m, s) in enumerate(picks):
        np.testing.assert_array_equal(got[:, k], full[m][:, s])


def test_randomized_with_one_bundle_is_deterministic():
    p = inputs.tiny_problem(21, R=7, S=[4, 6, 5])
    cost, q = blocks(p)
    a = O.mam(cost, q, 1.0, iters=30)
    b = O.mam(cost, q, 1.0, iters=30, bundles=[[0, 1, 2]], seq=[0] * 30)
    assert np.array_equal(a["p_bar"], b["p_bar"])
    for x, y in zip(a["theta"], b["theta"]):
        assert np.array_equal(x, y)


def test_randomized_step_leaves_other_measures_alone():
    """A step with M^k = {1}: measures 0 and 2 keep their plans and marginals
    bitwise; measure 1 gets exactly the deterministic step's plan."""
    p = inputs.tiny_problem(22, R=6, S=[3, 5, 4], masses=[0.8, 1.0, 1.2], gamma=0.1)
    cost, q = blocks(p)
    r = O.mam(cost, q, 1.0, p.gamma, iters=3)
    th, pm = r["theta"], r["pm"]
    det, pm_det, _ = O.mam_step(th, pm, cost, q, 1.0, p.gamma)
    ran, pm_ran, _ = O.mam_step(th, pm, cost, q, 1.0, p.gamma, chosen=[1])
    assert np.array_equal(ran[0], th[0]) and np.array_equal(ran[2], th[2])
    assert np.array_equal(pm_ran[0], pm[0]) and np.array_equal(pm_ran[2], pm[2])
    assert np.array_equal(ran[1], det[1]) and np.array_equal(pm_ran[1], pm_det[1])


def test_randomized_converges_to_lp_optimum():
    """Randomized MAM with single-measure bundles drawn with probability
    alpha_m = 1/M (Theorem on convergence, part b): the objective reaches the
    LP optimum of (HugeLP)."""
    p = inputs.tiny_problem(2, R=9, S=[5, 7, 6])
    cost, q = blocks(p)
    f_lp, _, _ = lp.wb_lp(cost, q)
    bundles = [[0], [1], [2]]
    seq = inputs.bundle_sequence(bundles, 12000, seed=1)
    r = O.mam(cost, q, 1.0, iters=12000, bundles=bundles, seq=seq)
    th = r["theta"]
    # pi_hat of the last full step from the final plans (every measure)
    _, _, info = O.mam_step(th, r["pm"], cost, q, 1.0, math.inf)
    d = O.diagnostics(cost, q, info["pi_hat"], th, th)
    assert abs(d["W_hat"] - f_lp) <= 1e-6 * max(1.0, abs(f_lp))
    assert abs(r["p_bar"].sum() - 1.0) < 1e-10
