"""Batches of independent problems and HIP-graph replay (MI355X only)."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def oracle_pbar(p, iters):
    return O.mam([p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)],
                 p.rho, p.gamma, iters)["p_bar"]


def mixed_batch(dtype):
    probs = [
        inputs.tiny_problem(1, R=81, S=[40, 23], dtype=dtype, zero_frac=0.1),
        inputs.tiny_problem(2, R=300, S=[17, 60, 5], dtype=dtype, shared=False),
        inputs.tiny_problem(3, R=64, S=[64, 64], dtype=dtype, shared=True),
        inputs.tiny_problem(4, R=1000, S=[12, 30], dtype=dtype, masses=[0.7, 1.3], gamma=0.05),
        inputs.balanced_sparse(K=12, M=4, dtype=dtype),
        inputs.tiny_problem(5, R=2000, S=[9, 14], dtype=dtype),
        inputs.unbalanced_dense(K=10, M=3, gamma=0.02, dtype=dtype),
        inputs.tiny_problem(6, R=5, S=[3, 1, 4], dtype=dtype),
    ]
    return probs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixed_batch_matches_oracle(dtype):
    probs = mixed_batch(dtype)
    b = mam.Batch(probs)
    say(f"batch of {len(probs)} problems, {b.groups()} shape groups: "
        f"{[b.schedule(g) for g in range(b.groups())]}")
    b.init()
    b.iterate(15)
    for i, p in enumerate(probs):
        got = b.barycenter(i).cpu().numpy()
        e = rel(got, oracle_pbar(p, 15))
        say(f"  {p.name} R={p.R} rel L1 {e:.3e}")
        assert e <= TOL[dtype]


def test_batched_config_shape_small():
    """Uneven R (k^2, k in 8..16), M in 2..8, S^m = R, FP32."""
    probs = inputs.batched_problems(n=12, k_range=(8, 16), iters=20)
    b = mam.Batch(probs)
    b.init()
    b.iterate(20)
    worst = max(rel(b.barycenter(i).cpu().numpy(), oracle_pbar(p, 20)) for i, p in enumerate(probs))
    say(f"worst rel L1 over 12 problems: {worst:.3e}")
    assert worst <= TOL["f32"]


def test_batch_graph_replays_equal_eager():
    probs = inputs.batched_problems(n=6, k_range=(8, 20), iters=30)
    eager = mam.Batch(probs)
    eager.init()
    graphed = mam.Batch(probs)
    graphed.graph(5)
    graphed.init()
    for rep in range(4):
        eager.iterate(7)
        graphed.iterate(7)          # one replay of 5 plus 2 direct iterations
        torch.cuda.synchronize()
        for i in range(len(probs)):
            a = eager.barycenter(i).cpu().numpy()
            g = graphed.barycenter(i).cpu().numpy()
            assert np.array_equal(a, g), (rep, i)
            for x, y in zip(eager.plans(i), graphed.plans(i)):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_problem_graph_equals_eager(dtype):
    p = inputs.balanced_plain(dtype=dtype) if dtype == "f64" else inputs.unbalanced_dense(K=12, M=6, dtype="f32")
    a = mam.solver_for(p)
    g = mam.solver_for(p)
    g.graph(10)
    a.init()
    g.init()
    for rep in range(3):
        a.iterate(25)
        g.iterate(25)
        torch.cuda.synchronize()
        assert np.array_equal(a.barycenter().cpu().numpy(), g.barycenter().cpu().numpy())
    assert rel(g.barycenter().cpu().numpy(), oracle_pbar(p, 75)) <= TOL[dtype]


def test_graph_with_diagnostics_last_iteration():
    """With diagnostics on, the last iteration runs outside the graph and
    the figures match an eager run."""
    p = inputs.tiny_problem(3, R=200, S=[30, 40], dtype="f64")
    a = mam.solver_for(p, diag=True)
    g = mam.solver_for(p, diag=True)
    g.graph(4)
    a.init()
    g.init()
    a.iterate(13)
    g.iterate(13)
    da, dg = a.diagnostics(), g.diagnostics()
    assert da == dg
