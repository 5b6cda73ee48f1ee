"""Pins of the FP64 gradient oracle (CPU only): its forward equals the numpy
oracle, and its gradients equal central finite differences of the numpy
oracle where no active set changes within +-h (the map is piecewise affine,
so central differences are exact there)."""
import numpy as np
import pytest

from oracle import mam_grad as G
from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def loss_np(cost, q, rho, iters, target):
    pb = O.mam(cost, q, rho, iters=iters)["p_bar"]
    return float(((pb - target) ** 2).sum())


@pytest.mark.parametrize("seed", range(3))
def test_forward_matches_numpy_oracle(seed):
    p = inputs.tiny_problem(seed, R=7, S=[5, 6, 4], zero_frac=0.2)
    cost, q = blocks(p)
    tgt = np.random.default_rng(seed).dirichlet(np.ones(7))
    L, pbar, _, _ = G.loss_and_grads(cost, q, 1.3, 12, tgt)
    np.testing.assert_allclose(pbar, O.mam(cost, q, 1.3, iters=12)["p_bar"], atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_gradients_match_central_differences(seed):
    p = inputs.tiny_problem(10 + seed, R=6, S=[4, 5], zero_frac=0.0)
    cost, q = blocks(p)
    rho, iters = 0.7, 8
    tgt = np.random.default_rng(seed).dirichlet(np.ones(6))
    _, _, gq, gc = G.loss_and_grads(cost, q, rho, iters, tgt)
    rng = np.random.default_rng(100 + seed)
    h = 1e-7
    checked = 0
    for trial in range(6):
        # q direction preserving the masses (balanced problems); c direction free
        du = [rng.normal(size=qm.shape) for qm in q]
        du = [d - d.mean() for d in du]
        dc = [rng.normal(size=c.shape) for c in cost]
        for which in ("q", "c"):
            if which == "q":
                plus = [qm + h * d for qm, d in zip(q, du)]
                minus = [qm - h * d for qm, d in zip(q, du)]
                if min(x.min() for x in minus) <= 0:
                    continue
                fd = (loss_np(cost, plus, rho, iters, tgt) - loss_np(cost, minus, rho, iters, tgt)) / (2 * h)
                an = sum(float((g * d).sum()) for g, d in zip(gq, du))
            else:
                plus = [c + h * d for c, d in zip(cost, dc)]
                minus = [c - h * d for c, d in zip(cost, dc)]
                fd = (loss_np(plus, q, rho, iters, tgt) - loss_np(minus, q, rho, iters, tgt)) / (2 * h)
                an = sum(float((g * d).sum()) for g, d in zip(gc, dc))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, fd, an)
            checked += 1
    assert checked >= 8
