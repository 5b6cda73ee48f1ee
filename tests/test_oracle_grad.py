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


@pytest.mark.parametrize("seed", range(3))
def test_vjp_is_the_adjoint_of_the_jvp(seed):
    """<J^T u, v> = <u, J v> with J v by central differences of the numpy
    oracle (exact for a piecewise-affine map away from kinks)."""
    p = inputs.tiny_problem(20 + seed, R=5, S=[4, 3, 5], zero_frac=0.0)
    cost, q = blocks(p)
    rho, iters = 1.1, 7
    rng = np.random.default_rng(200 + seed)
    u = rng.normal(size=5)
    pbar, gq, gc = G.vjp(cost, q, rho, iters, u)
    np.testing.assert_allclose(pbar, O.mam(cost, q, rho, iters=iters)["p_bar"], atol=1e-14)
    h = 1e-7
    dq = [rng.normal(size=x.shape) for x in q]
    dq = [d - d.mean() for d in dq]
    dc = [rng.normal(size=c.shape) for c in cost]
    fplus = O.mam([c + h * d for c, d in zip(cost, dc)], [x + h * d for x, d in zip(q, dq)], rho, iters=iters)["p_bar"]
    fminus = O.mam([c - h * d for c, d in zip(cost, dc)], [x - h * d for x, d in zip(q, dq)], rho, iters=iters)["p_bar"]
    jv = (fplus - fminus) / (2 * h)
    lhs = sum(float((g * d).sum()) for g, d in zip(gq, dq)) + sum(float((g * d).sum()) for g, d in zip(gc, dc))
    rhs = float(u @ jv)
    assert abs(lhs - rhs) <= 1e-6 * max(1.0, abs(rhs)), (lhs, rhs)


def test_vjp_of_the_loss_gradient():
    p = inputs.tiny_problem(31, R=6, S=[5, 5])
    cost, q = blocks(p)
    tgt = np.full(6, 1 / 6)
    L, pbar, gq, gc = G.loss_and_grads(cost, q, 1.0, 9, tgt)
    _, gq2, gc2 = G.vjp(cost, q, 1.0, 9, 2 * (pbar - tgt))
    for a, b in zip(gq + gc, gq2 + gc2):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-16)


def test_cost_gradient_columns_sum_to_zero():
    """Adding a constant to one cost column shifts w uniformly in that column
    and leaves its projection unchanged, so every column of dL/dc sums to 0."""
    p = inputs.tiny_problem(41, R=8, S=[6, 7])
    cost, q = blocks(p)
    _, _, _, gc = G.loss_and_grads(cost, q, 0.9, 10, np.random.default_rng(3).dirichlet(np.ones(8)))
    for g in gc:
        assert np.abs(g.sum(axis=0)).max() <= 1e-14 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("seed", range(3))
def test_unbalanced_forward_and_gradients(seed):
    """Finite gamma with the damping active (t < 1): forward equals the numpy
    oracle; gradients equal central differences (q moves freely: the masses
    need not stay equal)."""
    p = inputs.tiny_problem(50 + seed, R=6, S=[5, 4], masses=[0.7, 1.3], gamma=0.02)
    cost, q = blocks(p)
    rho, iters, gamma = 1.0, 8, p.gamma
    tgt = np.random.default_rng(seed).dirichlet(np.ones(6))
    ora = O.mam(cost, q, rho, gamma, iters, record=True)
    assert min(ora["hist"]["t"]) < 1.0
    _, pbar, gq, gc = G.loss_and_grads(cost, q, rho, iters, tgt, gamma)
    np.testing.assert_allclose(pbar, ora["p_bar"], atol=1e-14)
    rng = np.random.default_rng(300 + seed)
    h = 1e-7
    lossf = lambda c, qq: float(((O.mam(c, qq, rho, gamma, iters)["p_bar"] - tgt) ** 2).sum())
    for _ in range(3):
        du = [rng.normal(size=x.shape) * x for x in q]
        dc = [rng.normal(size=c.shape) for c in cost]
        fd = (lossf(cost, [x + h * d for x, d in zip(q, du)]) - lossf(cost, [x - h * d for x, d in zip(q, du)])) / (2 * h)
        an = sum(float((g * d).sum()) for g, d in zip(gq, du))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
        fd = (lossf([c + h * d for c, d in zip(cost, dc)], q) - lossf([c - h * d for c, d in zip(cost, dc)], q)) / (2 * h)
        an = sum(float((g * d).sum()) for g, d in zip(gc, dc))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
