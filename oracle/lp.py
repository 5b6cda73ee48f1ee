"""Brute-force references for tiny instances (TEST INFRASTRUCTURE ONLY).

* ``wb_lp``: the fixed-support barycenter LP (HugeLP) written out as plain
  constraints and handed to scipy's HiGHS solver.  The cost matrices are taken
  as given (the alpha_m factor of (HugeLP) is folded into c^(m), as in the
  splitting of Sec. 4 eq. (fm)).
* ``uwb_slsqp``: the unbalanced problem (UWB) -- transport cost plus
  gamma * dist_L over the product of the sets Pi^(m) -- minimised directly
  with scipy's SLSQP on instances with a few dozen variables; with
  ``relaxed`` the column sums are only bounded by q^(m)_s (the full
  unbalanced extension).

Only the test suite may import this module.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np
from scipy.optimize import linprog, minimize

__all__ = ["wb_lp", "uwb_objective", "uwb_slsqp"]


def wb_lp(cost: List[np.ndarray], q: List[np.ndarray]):
    """Solve (HugeLP): min sum_m <c^(m), pi^(m)> over p >= 0, pi^(m) >= 0 with
    sum_r pi^(m)_rs = q^(m)_s and sum_s pi^(m)_rs = p_r.

    Returns (objective, p, [pi^(m)]).
    """
    R = cost[0].shape[0]
    S = [c.shape[1] for c in cost]
    nvar = R + sum(R * s for s in S)
    obj = np.zeros(nvar)
    rows, rhs = [], []
    off = R
    offs = []
    for m, c in enumerate(cost):
        offs.append(off)
        obj[off:off + R * S[m]] = c.ravel()          # pi^(m)_rs at off + r*S + s
        for s in range(S[m]):                        # column sums = q_s
            row = np.zeros(nvar)
            row[off + np.arange(R) * S[m] + s] = 1.0
            rows.append(row)
            rhs.append(q[m][s])
        for r in range(R):                           # row sums = p_r
            row = np.zeros(nvar)
            row[off + r * S[m]: off + (r + 1) * S[m]] = 1.0
            row[r] = -1.0
            rows.append(row)
            rhs.append(0.0)
        off += R * S[m]
    res = linprog(obj, A_eq=np.array(rows), b_eq=np.array(rhs),
                  bounds=[(0, None)] * nvar, method="highs")
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    x = res.x
    pis = [x[o:o + R * s].reshape(R, s) for o, s in zip(offs, S)]
    return float(res.fun), x[:R].copy(), pis


def uwb_objective(cost: List[np.ndarray], pis: List[np.ndarray], gamma: float) -> float:
    """sum_m <c^(m), pi^(m)> + gamma * dist_L(pi), problem (UWB)."""
    S = [c.shape[1] for c in cost]
    inv = 1.0 / np.asarray(S, dtype=np.float64)
    a = inv / inv.sum()
    pm = np.stack([pi.sum(axis=1) for pi in pis])
    p = (a[:, None] * pm).sum(axis=0)
    d = math.sqrt(sum(float(((p - pm[m]) ** 2).sum()) / S[m] for m in range(len(S))))
    return sum(float((c * pi).sum()) for c, pi in zip(cost, pis)) + gamma * d


def uwb_slsqp(cost: List[np.ndarray], q: List[np.ndarray], gamma: float, x0=None,
              iters: int = 2000, relaxed: bool = False):
    """Minimise problem (UWB) over pi^(m) in Pi^(m) with SLSQP (tiny sizes);
    relaxed: over pi^(m) >= 0 with column sums <= q^(m)_s."""
    R = cost[0].shape[0]
    S = [c.shape[1] for c in cost]
    sizes = [R * s for s in S]
    offs = np.concatenate([[0], np.cumsum(sizes)])

    def unpack(x):
        return [x[offs[m]:offs[m + 1]].reshape(R, S[m]) for m in range(len(S))]

    def f(x):
        return uwb_objective(cost, unpack(x), gamma)

    cons = []
    for m in range(len(S)):
        for s in range(S[m]):
            idx = offs[m] + np.arange(R) * S[m] + s
            if relaxed:
                cons.append({"type": "ineq",
                             "fun": (lambda x, idx=idx, v=q[m][s]: v - x[idx].sum()),
                             "jac": (lambda x, idx=idx: -_unit(x.size, idx))})
            else:
                cons.append({"type": "eq",
                             "fun": (lambda x, idx=idx, v=q[m][s]: x[idx].sum() - v),
                             "jac": (lambda x, idx=idx: _unit(x.size, idx))})
    if x0 is None:
        x0 = np.concatenate([np.repeat((qm / R)[None, :], R, axis=0).ravel() for qm in q])
    res = minimize(f, x0, method="SLSQP", constraints=cons,
                   bounds=[(0, None)] * x0.size,
                   options={"maxiter": iters, "ftol": 1e-14})
    return float(res.fun), unpack(res.x)


def _unit(n, idx):
    g = np.zeros(n)
    g[idx] = 1.0
    return g
