"""Pins of the free-support workload generator (CPU only).

* Xi has ((K-1)M+1)^d points and holds every average of M pixel centres
  (Theorem c, item a, with alpha_m = 1/M);
* Theorem c, item c: the LP (HugeLP) over Xi reaches the same optimum as over
  a twice finer grid containing Xi, and beats the LP restricted to the pixel
  grid itself;
* the nested-ellipse images are histograms of mass 1 and the cost columns
  built from points are the squared distances.
"""
import itertools

import numpy as np
import pytest

from oracle import lp
from paper_2309_05315_amd import inputs


def test_grid_size_and_averages():
    for K, M in ((3, 2), (4, 3), (60, 10)):
        xi = inputs.free_support_grid(K, M)
        assert xi.shape == (((K - 1) * M + 1) ** 2, 2)
    assert inputs.free_support_grid(60, 10).shape[0] == 349281
    K, M = 4, 3
    xi = inputs.free_support_grid(K, M)
    c = (np.arange(K) + 0.5) / K
    rng = np.random.default_rng(0)
    pts = set(map(tuple, np.round(xi * M * K * 2).astype(int)))
    for _ in range(50):
        ij = rng.integers(0, K, size=(M, 2))
        avg = c[ij].mean(axis=0)
        assert tuple(np.round(avg * M * K * 2).astype(int)) in pts


def _lp_value(support, zeta, qs):
    cost = []
    for _ in qs:
        d = ((support[:, None, :] - zeta[None, :, :]) ** 2).sum(axis=2)
        cost.append(d / len(qs))  # alpha_m = 1/M folded into c^(m)
    val, _, _ = lp.wb_lp(cost, qs)
    return val


@pytest.mark.parametrize("seed", range(3))
def test_theorem_c_support_is_enough(seed):
    K, M = 3, 2
    rng = np.random.default_rng([31, seed])
    c = (np.arange(K) + 0.5) / K
    X, Y = np.meshgrid(c, c, indexing="ij")
    zeta = np.stack([X.ravel(), Y.ravel()], axis=1)
    qs = []
    for _ in range(M):
        w = rng.uniform(0, 1, K * K) * (rng.uniform(0, 1, K * K) < 0.6)
        w[rng.integers(K * K)] += 0.5
        qs.append(w / w.sum())
    xi = inputs.free_support_grid(K, M)
    v_xi = _lp_value(xi, zeta, qs)
    # a grid of twice the resolution that contains Xi
    n = M * (K - 1) + 1
    v = (np.arange(2 * n - 1) / 2 + M / 2) / (M * K)
    G = np.stack([g.ravel() for g in np.meshgrid(v, v, indexing="ij")], axis=1)
    v_fine = _lp_value(G, zeta, qs)
    v_pix = _lp_value(zeta, zeta, qs)
    assert v_xi == pytest.approx(v_fine, rel=1e-7, abs=1e-10)
    assert v_pix > v_xi * (1 + 1e-6)


def test_nested_ellipses_and_point_cost():
    p = inputs.free_support(seed=1, K=12, M=3, dtype="f64")
    assert p.R == (11 * 3 + 1) ** 2 and p.S == [144] * 3 and p.cost is None
    for m in range(p.M):
        qm = p.q_block(m)
        assert qm.min() >= 0 and abs(qm.sum() - 1) < 1e-12
    for cidx in (0, 57, 143):
        col = p.cost_column(cidx)
        brute = np.array([((x - p.zeta[cidx]) ** 2).sum() for x in p.xi])
        np.testing.assert_allclose(col, brute, rtol=1e-15, atol=0)
    blk = p.cost_block(2)
    assert blk.shape == (p.R, 144)
    np.testing.assert_array_equal(blk[:, 57], p.cost_column(57))


def test_grid_parameters_reproduce_xi_bitwise():
    # the kernels of the grid cost mode evaluate origin + i * spacing with the
    # same two rounded operations
    p = inputs.free_support(seed=0, K=12, M=3, dtype="f64")
    (n0, n1), (o0, o1), (h0, h1) = p.meta["grid"]
    assert n0 * n1 == p.R
    r = np.arange(p.R)
    i0, i1 = r // n1, r % n1
    np.testing.assert_array_equal(p.xi[:, 0], o0 + i0.astype(np.float64) * h0)
    np.testing.assert_array_equal(p.xi[:, 1], o1 + i1.astype(np.float64) * h1)
