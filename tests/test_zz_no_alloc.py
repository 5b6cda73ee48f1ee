"""mam_solve_static (one solve on the library's static device workspace, no
allocation) against the handle sequence it stands for (mam_create,
mam_set_workspace with a caller-allocated workspace, mam_bind, mam_init,
mam_iterate, mam_barycenter), bit for bit: two calls in a row on one GPU,
the second on a smaller problem, so the second runs on what the first left
in the shared array (MI355X only)."""
import sys

import numpy as np
import pytest
import torch

from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def by_handle(p, iters):
    s = mam.solver_for(p)
    s.init()
    s.iterate(iters)
    pb = s.barycenter().cpu().numpy()
    th = s.theta.cpu().numpy().copy()
    s.close()
    return pb, th


def by_static(p, iters):
    """The same buffers solver_for would bind, without a handle."""
    s = mam.solver_for(p)          # only to build the bound buffers and the layout
    theta = torch.zeros_like(s.theta)
    cost, q, idx = s.cost, s.q, s.index
    mode, ncols = s.cost_mode, s.cost_ncols
    s.close()
    pb = mam.solve_static(p.R, p.S, theta, cost, q, iters, rho=p.rho, gamma=p.gamma, cost_mode=mode,
                          index=idx, cost_ncols=ncols)
    return pb.cpu().numpy(), theta.cpu().numpy()


@pytest.mark.parametrize("order", ["large_first", "small_first"])
def test_static_solve_equals_handle_solve_twice(order):
    big = inputs.balanced_sparse(dtype="f32")                       # the benchmark workload, 67 MiB of workspace
    small = inputs.unbalanced_dense(K=12, M=5, gamma=0.02, dtype="f64")
    cases = [(big, 12), (small, 30)]
    if order == "small_first":
        cases = [(small, 30), (inputs.tiny_problem(3, R=130, S=[20, 7, 33], dtype="f32", zero_frac=0.1), 9)]
    for p, iters in cases:
        say(f"case {p.name} {p.dtype} R={p.R} M={p.M} T={p.T} iters={iters}")
        ref_pb, ref_th = by_handle(p, iters)
        pb, th = by_static(p, iters)
        torch.cuda.synchronize()
        assert np.array_equal(pb, ref_pb)
        assert np.array_equal(th, ref_th)
        assert np.isfinite(pb).all() and abs(pb.sum() - ref_pb.sum()) == 0.0
