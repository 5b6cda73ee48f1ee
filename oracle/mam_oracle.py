"""Plain FP64 CPU oracle of the Method of Averaged Marginals (MAM).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run this module.  The HIP library
never calls it, and it shares no code with the HIP library: it takes plain
arrays (cost blocks c^(m), weights q^(m)) and follows the paper's steps in the
paper's notation, one numpy statement per step, in float64, with no blocking,
fusion or reordering beyond what the paper itself writes.

Paper: Mimouni, Malisani, Zhu, de Oliveira, "Computing Wasserstein barycenter
via operator splitting: the method of averaged marginals" (arXiv 2309.05315).

Functions and the passage each follows:

* ``proj_simplex_sort``  Prop. 3 (eq. (proj-s)) and the Remark on Delta_R(tau):
  exact Euclidean projection onto {u >= 0, sum u = tau}; the exact
  sort-based threshold method that the paper delegates to (Condat 2016).
* ``proj_subsimplex``  the extension to the full unbalanced setting (the
  section on relaxing the marginals of q^(m) as well, and its proposition):
  projection onto {u >= 0, sum u <= tau} by clamping at 0 and, if the clamped
  vector carries more than tau, the simplex projection.
* ``marginals``, ``averaging_weights``, ``average``, ``proj_L``  Prop. 2 (eqs. (pr), (row_sol)).
* ``dist_L``, ``dist_L_marginals``  the reduction of dist_L to R-vectors stated after Alg. 1.
* ``unbalanced_prox``  eq. (Unbalanced-prox).
* ``damping``  the t^k rule of Alg. 1 (Step 1).
* ``mam``  Alg. 1 with the deterministic choice M^k = {1, ..., M}.
* ``mam_step_columns``  Step 2 of Alg. 1 for a sample of columns (exact,
  since the columns are independent given the marginals, Prop. 3).
* ``diagnostics``  the stopping quantities of Sec. 5 (Stopping criteria) and
  the objective/feasibility figures used in Sec. 6.3.
* ``mam_until``  Alg. 1 with one of the stopping tests of Sec. 5 (Stopping
  criteria) evaluated every few iterations in place of "while not converged".
* ``support_update``  the support step of the fixed-support approach (Sec. 2,
  the alternation between the LP on a fixed support and the support problem
  with the plans fixed) in the closed form of the free-support proposition
  (Prop. 4): each point is the alpha-weighted mean of the measures' points,
  weighted by the mass the plans carry from it.
* ``free_support_alternation``  the alternating method of that section
  (Alg. 2): the cost alpha_m/2 ||xi_r - zeta_s||^2 on the current support,
  Alg. 1 on it, then the support step on the plans of its last iteration.

Readings where the paper is silent or loose:

* theta^0_rs = q_s / R (Alg. 1 leaves theta^0 arbitrary);
* the returned barycenter is sum_m a_m p^(m) of the final theta^K (Alg. 1
  returns p^k without advancing k: one more Step 1 is taken);
* a zero weight q_s = 0 gives the zero column (Remark on Delta_R(tau));
* when tau is below the rounding resolution of w, the threshold index j* is
  clamped to 1, so the column becomes 0 (the sort formula's own result in
  floating point, stated explicitly so it never divides by zero);
* the plans of the support step are the projections pi_hat^(m) of the last
  iteration's Step 2 (non-negative, column sums q_s); a point whose row
  carries no mass keeps its place (the formula's denominator is 0 there);
* in the alternation, Alg. 1 starts from theta^0 = q_s/R once and each later
  round continues from the plans of the previous one.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

__all__ = [
    "proj_simplex_sort",
    "proj_subsimplex",
    "averaging_weights",
    "average",
    "marginals",
    "proj_L",
    "dist_L",
    "dist_L_marginals",
    "unbalanced_prox",
    "damping",
    "mam_step",
    "mam_step_columns",
    "mam",
    "diagnostics",
    "mam_until",
    "STOP_TESTS",
    "sq_euclid_cost",
    "support_update",
    "free_support_alternation",
]


# ---------------------------------------------------------------------------
# Prop. 3 / Remark: projection onto the scaled simplex Delta_R(tau)
# ---------------------------------------------------------------------------
def proj_simplex_sort(w: np.ndarray, tau) -> tuple:
    """Project every column of ``w`` (R x n) onto Delta_R(tau_s).

    Sort-based exact method: with u the column sorted in decreasing order,
    j* = max{ j : u_j > (sum_{i<=j} u_i - tau) / j },
    lambda = (sum_{i<=j*} u_i - tau) / j*,  result = max(w - lambda, 0).
    A column with tau_s = 0 projects to 0 (Delta_R(0) = {0}).

    Returns (pi_hat, lam) with lam = +inf for tau_s = 0 columns.
    """
    w = np.asarray(w, dtype=np.float64)
    if w.ndim == 1:
        p, lam = proj_simplex_sort(w[:, None], np.atleast_1d(tau))
        return p[:, 0], lam[0]
    R, n = w.shape
    tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (n,))
    out = np.zeros_like(w)
    lam = np.full(n, np.inf)
    pos = tau > 0
    if not np.any(pos):
        return out, lam
    wp = w[:, pos]
    tp = tau[pos]
    u = -np.sort(-wp, axis=0)                   # decreasing
    cs = np.cumsum(u, axis=0)
    j = np.arange(1, R + 1, dtype=np.float64)[:, None]
    cond = u > (cs - tp[None, :]) / j
    # j* = largest j with cond true (cond holds on a prefix); clamp to 1.
    last_true = R - 1 - np.argmax(cond[::-1, :], axis=0)
    any_true = cond.any(axis=0)
    jstar = np.where(any_true, last_true + 1, 1)
    cols = np.arange(wp.shape[1])
    lam_p = (cs[jstar - 1, cols] - tp) / jstar
    out[:, pos] = np.maximum(wp - lam_p[None, :], 0.0)
    lam[pos] = lam_p
    return out, lam


# ---------------------------------------------------------------------------
# Prop. 2: projection onto the subspace L of balanced plans
# ---------------------------------------------------------------------------
def proj_subsimplex(w: np.ndarray, tau) -> np.ndarray:
    """Project every column of ``w`` (R x n) onto {u >= 0, sum u <= tau_s}:
    first u = max(w, 0); a column whose u sums to at most tau_s keeps it,
    any other column is projected onto Delta_R(tau_s) (the full unbalanced
    extension; tau_s = 0 gives 0)."""
    w = np.asarray(w, dtype=np.float64)
    tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), (w.shape[1],))
    out = np.maximum(w, 0.0)
    over = out.sum(axis=0) > tau
    if np.any(over):
        ph, _ = proj_simplex_sort(w[:, over], tau[over])
        out[:, over] = ph
    return out


def averaging_weights(S: Sequence[int]) -> np.ndarray:
    """a_m = (1/S^m) / sum_j (1/S^j), eq. (pr)."""
    inv = 1.0 / np.asarray(S, dtype=np.float64)
    return inv / inv.sum()


def marginals(theta: List[np.ndarray]) -> np.ndarray:
    """p^(m)_r = sum_s theta^(m)_rs, eq. (pr); returns an M x R array."""
    return np.stack([th.sum(axis=1) for th in theta])


def proj_L(theta: List[np.ndarray]):
    """Prop. 2: pi^(m)_rs = theta^(m)_rs + (p_r - p^(m)_r) / S^m.

    Returns (pi, p, pm) with p = sum_m a_m p^(m) and pm the M x R marginals.
    """
    S = [th.shape[1] for th in theta]
    a = averaging_weights(S)
    pm = marginals(theta)
    p = (a[:, None] * pm).sum(axis=0)
    pi = [th + ((p - pm[m]) / S[m])[:, None] for m, th in enumerate(theta)]
    return pi, p, pm


def average(pm: np.ndarray, S: Sequence[int]) -> np.ndarray:
    """p = sum_m a_m p^(m), eq. (pr) (Alg. 1, Step 1)."""
    a = averaging_weights(S)
    return (a[:, None] * pm).sum(axis=0)


def dist_L_marginals(pm: np.ndarray, S: Sequence[int]) -> float:
    """dist_L of plans whose row sums are ``pm`` (M x R): by Prop. 2 the
    distance depends on the plans only through their marginals,
    sqrt(sum_m ||p - p^(m)||^2 / S^m) with p = sum_m a_m p^(m) (text after Alg. 1)."""
    p = average(pm, S)
    return math.sqrt(sum(float(((p - pm[m]) ** 2).sum()) / S[m] for m in range(len(S))))


def dist_L(theta: List[np.ndarray]) -> float:
    """dist_L(theta) = sqrt(sum_m ||p - p^(m)||^2 / S^m) (text after Alg. 1)."""
    return dist_L_marginals(marginals(theta), [th.shape[1] for th in theta])


def unbalanced_prox(theta: List[np.ndarray], rho: float, gamma: float) -> List[np.ndarray]:
    """eq. (Unbalanced-prox): prox of gamma * dist_L with parameter rho."""
    pi, _, _ = proj_L(theta)
    d = dist_L(theta)
    if math.isinf(gamma) or rho * d <= gamma:
        return pi
    t = gamma / (rho * d)
    return [th + t * (pl - th) for th, pl in zip(theta, pi)]


def damping(p: np.ndarray, pm: np.ndarray, S: Sequence[int], rho: float, gamma: float):
    """Alg. 1, Step 1: t = 1 if rho * sqrt(sum_m ||p - p^(m)||^2 / S^m) <= gamma,
    else gamma / (rho * sqrt(...)).  gamma = inf is the balanced case."""
    d = math.sqrt(sum(float(((p - pm[m]) ** 2).sum()) / S[m] for m in range(len(S))))
    if math.isinf(gamma) or rho * d <= gamma:
        return 1.0, d
    return gamma / (rho * d), d


# ---------------------------------------------------------------------------
# Alg. 1 (deterministic MAM)
# ---------------------------------------------------------------------------
def mam_step(theta: List[np.ndarray], pm: np.ndarray, cost: List[np.ndarray],
             q: List[np.ndarray], rho: float, gamma: float, chosen: Optional[Sequence[int]] = None,
             relaxed: bool = False):
    """One pass of Alg. 1's loop body with M^k = {1, ..., M}, or with
    M^k = ``chosen`` (the randomized variant, eq. (DR-random)): Step 1 still
    averages every marginal, Steps 2 and 3 run only for the chosen measures,
    and every other plan and marginal is left as it was.

    Step 1: p^k = sum_m a_m p^(m); t^k from the damping rule.
    Step 2 (every m, every column s, all with the marginal p^(m) of theta^k):
        w      = theta^(m)_{:,s} + 2 t^k (p^k - p^(m)) / S^m - c^(m)_{:,s} / rho
        pi_hat = Proj_{Delta_R(q_s)}(w)
        theta' = pi_hat - t^k (p^k - p^(m)) / S^m
    Step 3: p^(m) = row sums of the new theta^(m).
    With ``relaxed`` the columns are projected onto {u >= 0, sum u <= q_s}
    instead (the full unbalanced extension; the cost passed is then the
    shifted d^(m) = c^(m) - eta).

    Returns (theta_new, pm_new, info) where info holds p^k, t^k, the
    distance d^k and the pi_hat blocks.
    """
    S = [th.shape[1] for th in theta]
    M = len(S)
    p = average(pm, S)                                    # Step 1
    t, d = damping(p, pm, S, rho, gamma)
    active = set(range(M)) if chosen is None else set(int(m) for m in chosen)
    new_theta, pi_hat = [], []
    for m in range(M):                                    # Step 2
        if m not in active:
            pi_hat.append(None)
            new_theta.append(theta[m])
            continue
        corr = t * (p - pm[m]) / S[m]
        w = theta[m] + 2.0 * corr[:, None] - cost[m] / rho
        ph = proj_subsimplex(w, q[m]) if relaxed else proj_simplex_sort(w, q[m])[0]
        pi_hat.append(ph)
        new_theta.append(ph - corr[:, None])
    pm_new = pm.copy()                                    # Step 3
    for m in active:
        pm_new[m] = new_theta[m].sum(axis=1)
    return new_theta, pm_new, {"p": p, "t": t, "d": d, "pi_hat": pi_hat}


def mam_step_columns(theta_cols: np.ndarray, measure_of_col: Sequence[int], pm: np.ndarray,
                     cost_cols: np.ndarray, q_cols: np.ndarray, S: Sequence[int],
                     rho: float, gamma: float):
    """Alg. 1 Step 2 for a chosen set of columns only.

    Given the marginals p^(m) of theta^k (M x R), every column is updated
    independently of the others (Prop. 3), so a sample of columns can be
    advanced exactly: column k belongs to measure measure_of_col[k] and has
    values theta_cols[:, k], cost cost_cols[:, k] and weight q_cols[k].
    Returns (theta' columns, pi_hat columns, t).
    """
    a = averaging_weights(S)
    p = (a[:, None] * pm).sum(axis=0)
    t, _ = damping(p, pm, S, rho, gamma)
    new, ph_all = [], []
    for k, m in enumerate(measure_of_col):
        corr = t * (p - pm[m]) / S[m]
        w = theta_cols[:, k] + 2.0 * corr - cost_cols[:, k] / rho
        ph, _ = proj_simplex_sort(w[:, None], np.asarray(q_cols[k:k + 1], dtype=np.float64))
        ph_all.append(ph[:, 0])
        new.append(ph[:, 0] - corr)
    return np.stack(new, axis=1), np.stack(ph_all, axis=1), t


def mam(cost: List[np.ndarray], q: List[np.ndarray], rho: float,
        gamma: float = math.inf, iters: int = 1,
        theta0: Optional[List[np.ndarray]] = None, record: bool = False,
        bundles: Optional[Sequence[Sequence[int]]] = None, seq: Optional[Sequence[int]] = None,
        relaxed: bool = False) -> Dict:
    """Run Alg. 1 for ``iters`` iterations from theta^0.

    Randomized variant: with ``bundles`` (a partition of the measures, as in
    the remark on bundles) and ``seq`` (the bundle drawn at each iteration,
    supplied by the caller), iteration k uses M^k = bundles[seq[k]].

    cost[m]: R x S^m cost matrix c^(m) (taken as given, Sec. 4 eq. (fm));
    q[m]: weights q^(m) (length S^m); rho > 0; gamma in [0, inf].
    theta^0_rs = q_s / R unless ``theta0`` is given.

    Returns a dict with ``p_bar`` (= sum_m a_m p^(m) of theta^K), ``theta``,
    ``pm``, the last ``pi_hat``, the last ``t`` and, if ``record``, the
    per-iteration t, d and p histories.
    """
    cost = [np.asarray(c, dtype=np.float64) for c in cost]
    q = [np.asarray(v, dtype=np.float64) for v in q]
    R = cost[0].shape[0]
    S = [c.shape[1] for c in cost]
    if theta0 is None:
        theta = [np.repeat((qm / R)[None, :], R, axis=0) for qm in q]
    else:
        theta = [np.array(th, dtype=np.float64, copy=True) for th in theta0]
    pm = marginals(theta)                                 # Step 0
    hist = {"t": [], "d": [], "p": []}
    info = {"pi_hat": None, "t": None, "p": None}
    for k in range(iters):
        chosen = None if bundles is None else bundles[int(seq[k])]
        theta, pm_new, info = mam_step(theta, pm, cost, q, rho, gamma, chosen, relaxed)
        if record:
            hist["t"].append(info["t"])
            hist["d"].append(info["d"])
            hist["p"].append(info["p"])
        info["pm_old"] = pm
        pm = pm_new
    p_bar = average(pm, S)
    out = {"p_bar": p_bar, "theta": theta, "pm": pm, "pi_hat": info["pi_hat"],
           "t": info["t"], "p_prev": info["p"], "pm_prev": info.get("pm_old")}
    if record:
        out["hist"] = hist
    return out


# ---------------------------------------------------------------------------
# Diagnostics (stopping tests of Sec. 5; objective of Sec. 6.3)
# ---------------------------------------------------------------------------
def diagnostics(cost: List[np.ndarray], q: List[np.ndarray], pi_hat: List[np.ndarray],
                theta_new: List[np.ndarray], theta_old: List[np.ndarray]) -> Dict:
    """Figures reported for the last iteration.

    W_hat       = sum_m <c^(m), pi_hat^(m)> (the plan objective);
    dist_L      = dist_L(pi_hat);
    meas_resid  = max_{m,s} |sum_r pi_hat^(m)_rs - q^(m)_s|;
    dtheta_inf  = ||theta^{k+1} - theta^k||_inf.
    """
    W = sum(float((c * ph).sum()) for c, ph in zip(cost, pi_hat))
    res = max(float(np.abs(ph.sum(axis=0) - qm).max()) for ph, qm in zip(pi_hat, q))
    dth = max(float(np.abs(a - b).max()) for a, b in zip(theta_new, theta_old))
    return {"W_hat": W, "dist_L": dist_L(pi_hat), "meas_resid": res, "dtheta_inf": dth}


STOP_TESTS = ("dtheta", "dp", "dist")


def mam_until(cost: List[np.ndarray], q: List[np.ndarray], rho: float, max_iters: int,
              test: str, tol: float, check_every: int = 1, gamma: float = math.inf) -> Dict:
    """Alg. 1 run until a stopping test of Sec. 5 holds, at most ``max_iters``
    iterations.  After iteration j (j = 1, 2, ...) with j a multiple of
    ``check_every`` the test is evaluated on that iteration, and the run stops
    as soon as its value is <= tol:

    * "dtheta": ||theta^{k+1} - theta^k||_inf over every plan entry;
    * "dp":     ||p^{k+1} - p^k||_2, p^k = sum_m a_m p^(m) of theta^k;
    * "dist":   dist_L(pi_hat^k), the distance of the projected plans to the
      balanced set (the test the paper calls heuristic).

    Returns a dict with ``iters`` (iterations run), ``converged``, ``values``
    (the test's value at every check, in order), ``p_bar``, ``theta``, ``pm``.
    """
    if test not in STOP_TESTS:
        raise ValueError(f"unknown stopping test {test!r}")
    if check_every < 1:
        raise ValueError("check_every must be >= 1")
    cost = [np.asarray(c, dtype=np.float64) for c in cost]
    q = [np.asarray(v, dtype=np.float64) for v in q]
    R = cost[0].shape[0]
    S = [c.shape[1] for c in cost]
    a = averaging_weights(S)
    theta = [np.repeat((qm / R)[None, :], R, axis=0) for qm in q]
    pm = marginals(theta)
    values: List[float] = []
    converged = False
    j = 0
    while j < max_iters:
        theta_new, pm_new, info = mam_step(theta, pm, cost, q, rho, gamma)
        j += 1
        if j % check_every == 0:
            if test == "dtheta":
                v = max(float(np.abs(tn - to).max()) for tn, to in zip(theta_new, theta))
            elif test == "dp":
                p_new = (a[:, None] * pm_new).sum(axis=0)
                v = float(np.sqrt(((p_new - info["p"]) ** 2).sum()))
            else:
                v = dist_L(info["pi_hat"])
            values.append(v)
            converged = v <= tol
        theta, pm = theta_new, pm_new
        if converged:
            break
    p_bar = (a[:, None] * pm).sum(axis=0)
    return {"iters": j, "converged": converged, "values": values, "p_bar": p_bar, "theta": theta, "pm": pm}


def sq_euclid_cost(xi: np.ndarray, zeta: np.ndarray, normalize_max: bool = False) -> np.ndarray:
    """c_rs = ||xi_r - zeta_s||^2 (the cost of (HugeLP)), optionally / max."""
    xi = np.asarray(xi, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    c = np.zeros((xi.shape[0], zeta.shape[0]))
    for k in range(xi.shape[1]):
        c += (xi[:, k][:, None] - zeta[:, k][None, :]) ** 2
    if normalize_max:
        c = c / c.max()
    return c


def support_update(pi: List[np.ndarray], zeta: List[np.ndarray], alpha: Sequence[float],
                   xi_old: np.ndarray) -> Dict:
    """The support problem with the plans fixed, solved in closed form
    (Prop. 4; Sec. 2, the fixed-support approach):

        xi_r = sum_m alpha_m sum_s pi^(m)_rs zeta^(m)_s / sum_m alpha_m sum_s pi^(m)_rs,

    the minimiser of Psi(xi) = sum_m alpha_m sum_{r,s} 1/2 ||xi_r - zeta^(m)_s||^2 pi^(m)_rs.
    pi[m]: R x S^m plan; zeta[m]: S^m x d points; alpha: M weights; xi_old:
    R x d.  A row with no mass (denominator 0) keeps xi_old[r].
    Returns {"xi": R x d, "mass": the denominators (R)}.
    """
    xi_old = np.asarray(xi_old, dtype=np.float64)
    num = np.zeros_like(xi_old)
    den = np.zeros(xi_old.shape[0])
    for m in range(len(pi)):
        P = np.asarray(pi[m], dtype=np.float64)
        Z = np.asarray(zeta[m], dtype=np.float64)
        num += alpha[m] * (P @ Z)
        den += alpha[m] * P.sum(axis=1)
    xi = xi_old.copy()
    has = den > 0
    xi[has] = num[has] / den[has][:, None]
    return {"xi": xi, "mass": den}


def free_support_alternation(xi0: np.ndarray, zeta: List[np.ndarray], q: List[np.ndarray],
                             alpha: Sequence[float], rho: float, gamma: float = math.inf,
                             outer: int = 1, inner: int = 1) -> Dict:
    """The alternating method for the free-support barycenter (Alg. 2; Sec. 2):
    for k = 0, ..., outer - 1
        c^(m)_rs = alpha_m * 1/2 ||xi^k_r - zeta^(m)_s||^2   (the cost of (HugeLP) with
                                                         the weights alpha_m)
        ``inner`` iterations of Alg. 1 on that support (from theta^0 = q_s/R
        at k = 0, then from the previous round's plans)
        xi^{k+1} = support_update(pi_hat of the last iteration).
    Returns {"xi": the supports xi^1..xi^outer, "p_bar": the barycenter
    weights of each round, "theta": the final plans}.
    """
    xi = np.asarray(xi0, dtype=np.float64)
    theta = None
    xis, pbs = [], []
    for _ in range(outer):
        cost = [alpha[m] * 0.5 * sq_euclid_cost(xi, zeta[m]) for m in range(len(zeta))]
        out = mam(cost, q, rho, gamma, inner, theta0=theta)
        theta = out["theta"]
        xi = support_update(out["pi_hat"], zeta, alpha, xi)["xi"]
        xis.append(xi)
        pbs.append(out["p_bar"])
    return {"xi": xis, "p_bar": pbs, "theta": theta}
