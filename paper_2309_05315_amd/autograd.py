"""Differentiable MAM barycenter: torch.autograd.Function over the HIP
library's forward (mam_record) and hand-written reverse sweep (mam_backward).

    p_bar = barycenter(cost, q, S, rho=1.0, iters=100)

cost: (ncols, R) tensor (row k = cost column k); q: (T,) weights of the M
measures concatenated; S: columns per measure; gamma: the unbalanced
penalty (inf: balanced, equal masses).  Gradients flow to cost and q; p_bar
is float64 (R,).  The iteration starts from theta^0 = q/R.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import torch

from . import mam

__all__ = ["MAMBarycenter", "barycenter"]


class MAMBarycenter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, q, S, rho, gamma, iters, cost_mode, index, ckpt_every, schedule):
        ncols, R = cost.shape
        s = mam.Solver(R, S, rho=rho, gamma=gamma, dtype=cost.dtype, cost_mode=cost_mode, cost_ncols=ncols,
                       device=cost.device, **(schedule or {}))
        if s.cost_ld == R and cost.is_contiguous():
            cbuf = cost.detach()
        else:
            cbuf = torch.zeros(ncols, s.cost_ld, dtype=cost.dtype, device=cost.device)
            cbuf[:, :R] = cost.detach()
        theta = torch.empty(s.T, s.ld, dtype=cost.dtype, device=cost.device)
        s.bind(theta, cbuf, q.detach().contiguous(), index)
        s.init()
        s.record(iters, ckpt_every)
        ctx.solver = s
        ctx.R = R
        ctx.save_for_backward(cost, q)  # in-place changes before backward are reported by autograd
        return s.barycenter()

    @staticmethod
    def backward(ctx, grad_p):
        ctx.saved_tensors  # version check of cost and q
        gq, gc = ctx.solver.backward(grad_p)
        return gc[:, :ctx.R], gq, None, None, None, None, None, None, None, None


def barycenter(cost: torch.Tensor, q: torch.Tensor, S: Sequence[int], rho: float = 1.0,
               iters: int = 100, cost_mode: int = mam.COST_SHARED, gamma: float = math.inf,
               index: Optional[torch.Tensor] = None, ckpt_every: int = 0,
               schedule: Optional[dict] = None) -> torch.Tensor:
    """Barycenter after 'iters' MAM iterations, differentiable in cost and q.
    ckpt_every = C > 0 keeps theta every C iterations and recomputes windows
    in the backward pass; 0 keeps the active sets of every iteration."""
    return MAMBarycenter.apply(cost, q, [int(x) for x in S], float(rho), float(gamma), int(iters), int(cost_mode),
                               index, int(ckpt_every), schedule)
