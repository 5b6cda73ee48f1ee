"""Pins of the synthetic workload generator (CPU only)."""
import numpy as np

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs


def test_grid_cost_closed_form():
    """On a K x K pixel-centre grid, ||xi_r - xi_s||^2 scaled to max 1 equals
    (di^2 + dj^2) / (2 (K-1)^2), independent of the grid offset."""
    for K in (4, 16, 64):
        c = inputs.grid_cost(K)
        i, j = np.divmod(np.arange(K * K), K)
        ref = ((i[:, None] - i[None, :]) ** 2 + (j[:, None] - j[None, :]) ** 2) / (2.0 * (K - 1) ** 2)
        np.testing.assert_allclose(c, ref, atol=1e-15)
        # the oracle's plain cost definition gives the same matrix
        pts = inputs.grid_points(K)
        np.testing.assert_allclose(O.sq_euclid_cost(pts, pts, normalize_max=True), ref, atol=1e-15)


def test_problem_shapes_and_masses():
    p = inputs.balanced_plain()
    assert (p.R, p.M, p.T) == (256, 4, 1024) and p.shared_cost
    for m in range(p.M):
        assert abs(p.q_block(m).sum() - 1.0) < 1e-14
    p2 = inputs.balanced_sparse()
    assert p2.R == 4096 and p2.M == 32
    assert min(p2.S) > 500 and max(p2.S) <= 4096
    assert p2.col_index.dtype == np.int32 and p2.col_index.size == p2.T
    # f32 inputs are exactly representable in float32
    assert np.array_equal(p2.q.astype(np.float32).astype(np.float64), p2.q)
    p3 = inputs.unbalanced_dense(M=5)
    masses = [p3.q_block(m).sum() for m in range(5)]
    assert all(0.49 < x < 1.51 for x in masses)


def test_seeded_determinism():
    a = inputs.balanced_sparse(seed=3, K=16, M=4)
    b = inputs.balanced_sparse(seed=3, K=16, M=4)
    assert np.array_equal(a.q, b.q) and np.array_equal(a.col_index, b.col_index)
