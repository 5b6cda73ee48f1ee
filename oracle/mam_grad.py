"""FP64 CPU oracle of gradients through the MAM iteration (TEST INFRASTRUCTURE ONLY).

Alg. 1 (deterministic, balanced or unbalanced) written with torch CPU float64 tensors so
that autograd differentiates the unrolled iteration: theta^0 = q/R, K
iterations of Step 1 (average the marginals), Step 2 (reflect, project every
column onto Delta_R(q_s) by the sort-based exact formula of Prop. 3) and
Step 3 (new marginals), then the barycenter p-bar = sum_m a_m p^(m) of
theta^K.  The sort-based projection is piecewise affine in (w, q_s), so
autograd yields the exact derivative away from changes of the active set.

Only the test suite imports this module; it shares no code with the HIP
library and is pinned by tests against the numpy oracle (values) and
central finite differences of it (derivatives).
"""
from __future__ import annotations

import math
from typing import List

import numpy as np
import torch

__all__ = ["proj_simplex_sort_t", "mam_pbar_t", "loss_and_grads", "vjp"]


def proj_simplex_sort_t(w: torch.Tensor, tau: torch.Tensor) -> torch.Tensor:
    """Project every column of w (R x n) onto Delta_R(tau_s) (Prop. 3):
    with u the column sorted decreasingly, j* = max{j : u_j > (sum_{i<=j} u_i - tau)/j},
    lambda = (sum_{i<=j*} u_i - tau)/j*, result max(w - lambda, 0); tau_s = 0 gives 0."""
    R = w.shape[0]
    u, _ = torch.sort(w, dim=0, descending=True)
    cs = torch.cumsum(u, dim=0)
    j = torch.arange(1, R + 1, dtype=w.dtype).unsqueeze(1)
    cond = u > (cs - tau.unsqueeze(0)) / j
    jstar = torch.where(cond, j.expand_as(cond), torch.zeros_like(j).expand_as(cond)).amax(dim=0)
    jstar = torch.clamp(jstar, min=1).long()
    lam = (cs.gather(0, (jstar - 1).unsqueeze(0)).squeeze(0) - tau) / jstar.to(w.dtype)
    out = torch.clamp(w - lam.unsqueeze(0), min=0.0)
    return torch.where(tau.unsqueeze(0) > 0, out, torch.zeros_like(out))


def mam_pbar_t(cost: List[torch.Tensor], q: List[torch.Tensor], rho: float, iters: int,
               gamma: float = math.inf) -> torch.Tensor:
    """Barycenter after 'iters' MAM iterations from theta^0 = q/R.  With a
    finite gamma, Step 1's damping t^k = min(1, gamma / (rho d^k)), d^k =
    sqrt(sum_m ||p - p^(m)||^2 / S^m) (eq. (Unbalanced-prox)), scales the
    correction b^(m) = t^k (p - p^(m)) / S^m and is differentiated like the rest."""
    R = cost[0].shape[0]
    S = [c.shape[1] for c in cost]
    inv = torch.tensor([1.0 / s for s in S], dtype=torch.float64)
    a = inv / inv.sum()
    theta = [qm.unsqueeze(0).expand(R, -1) / R for qm in q]
    pm = torch.stack([th.sum(dim=1) for th in theta])
    for _ in range(iters):
        p = (a.unsqueeze(1) * pm).sum(dim=0)
        t = torch.ones((), dtype=torch.float64)
        if not math.isinf(gamma):
            d = torch.sqrt(sum(((p - pm[m]) ** 2).sum() / S[m] for m in range(len(S))))
            if float((rho * d).detach()) > gamma:
                t = gamma / (rho * d)
        new = []
        for m in range(len(S)):
            corr = t * (p - pm[m]) / S[m]
            w = theta[m] + 2.0 * corr.unsqueeze(1) - cost[m] / rho
            new.append(proj_simplex_sort_t(w, q[m]) - corr.unsqueeze(1))
        theta = new
        pm = torch.stack([th.sum(dim=1) for th in theta])
    return (a.unsqueeze(1) * pm).sum(dim=0)


def _grad(x: torch.Tensor):
    """x.grad as numpy; zeros when x took no part (the cost with 0 iterations)."""
    return np.zeros(tuple(x.shape)) if x.grad is None else x.grad.numpy().copy()


def loss_and_grads(cost_np, q_np, rho, iters, target_np, gamma=math.inf):
    """L = ||p-bar - target||^2 and its gradients with respect to every q^(m)
    and every c^(m) (lists of numpy arrays, float64)."""
    cost = [torch.tensor(c, dtype=torch.float64, requires_grad=True) for c in cost_np]
    q = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in q_np]
    pbar = mam_pbar_t(cost, q, rho, iters, gamma)
    loss = ((pbar - torch.tensor(target_np, dtype=torch.float64)) ** 2).sum()
    loss.backward()
    return (float(loss.detach()), pbar.detach().numpy(), [_grad(v) for v in q], [_grad(c) for c in cost])


def vjp(cost_np, q_np, rho, iters, u_np, gamma=math.inf):
    """p-bar and the vector-Jacobian products u^T dp-bar/dq^(m), u^T dp-bar/dc^(m)."""
    cost = [torch.tensor(c, dtype=torch.float64, requires_grad=True) for c in cost_np]
    q = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in q_np]
    pbar = mam_pbar_t(cost, q, rho, iters, gamma)
    pbar.backward(torch.tensor(u_np, dtype=torch.float64))
    return pbar.detach().numpy(), [_grad(v) for v in q], [_grad(c) for c in cost]
