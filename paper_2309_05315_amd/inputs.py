"""Seeded synthetic workloads for fixed-support Wasserstein barycenters.

The paper measures MAM on image histograms (MNIST digits, nested ellipses,
letters: Sec. 6).  None of those datasets is available here, so every workload
is a K x K pixel histogram drawn from a mixture of 1-3 isotropic Gaussian
blobs, with the barycenter and the measures on pixel-centre grids of [0,1]^2
and the squared Euclidean cost of the LP (HugeLP) scaled to maximum 1.

This module only produces inputs (support points, weights, cost columns).  It
holds no step of the method and imports nothing from the rest of the package,
so the HIP path and the CPU oracle can both consume what it returns.

Layout conventions shared by every consumer:

* plan columns are numbered globally j = off_m + s (measure m, column s of
  measure m), measures in order; T = sum_m S^m;
* ``cost`` has shape (ncols, R): row k is one cost column of length R
  (column-major storage of an R x ncols matrix);
* ``col_index`` (int32, length T) names the cost column of plan column j; it
  is ``None`` for a shared cost (plan column (m, s) uses cost column s);
* ``q`` has length T: the weights q^(m)_s of every measure, concatenated.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Problem",
    "grid_points",
    "sq_euclid",
    "grid_cost",
    "blob_density",
    "balanced_plain",
    "balanced_sparse",
    "unbalanced_dense",
    "adjoint_problem",
    "batched_problems",
    "tiny_problem",
    "line_problem",
    "free_support_grid",
    "free_support_axis",
    "nested_ellipses",
    "free_support",
]


@dataclass
class Problem:
    """One fixed-support barycenter instance (inputs only)."""

    name: str
    R: int
    S: List[int]
    cost: np.ndarray              # (ncols, R) float64 (already rounded to dtype)
    q: np.ndarray                 # (T,) float64 (already rounded to dtype)
    col_index: Optional[np.ndarray] = None   # (T,) int32, or None = shared
    rho: float = 1.0
    gamma: float = float("inf")
    iters: int = 1
    dtype: str = "f64"            # storage precision of plans, cost, q
    meta: dict = field(default_factory=dict)
    # support points instead of a stored cost (cost None): c_rs = ||xi_r - zeta_s||^2
    xi: Optional[np.ndarray] = None      # (R, d) float64
    zeta: Optional[np.ndarray] = None    # (ncols, d) float64

    @property
    def M(self) -> int:
        return len(self.S)

    @property
    def T(self) -> int:
        return int(sum(self.S))

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.S)]).astype(np.int64)

    @property
    def shared_cost(self) -> bool:
        return self.col_index is None

    def cost_columns(self, m: int) -> np.ndarray:
        """Indices into ``cost`` of the S^m columns of measure m."""
        off = self.offsets
        if self.col_index is None:
            return np.arange(self.S[m])
        return self.col_index[off[m]:off[m + 1]].astype(np.int64)

    def cost_block(self, m: int) -> np.ndarray:
        """c^(m) as an R x S^m float64 matrix."""
        if self.cost is None:
            return np.stack([self.cost_column(int(c)) for c in self.cost_columns(m)], axis=1)
        return np.ascontiguousarray(self.cost[self.cost_columns(m)].T)

    @property
    def cost_ncols(self) -> int:
        return int(self.zeta.shape[0] if self.cost is None else self.cost.shape[0])

    def cost_column(self, c: int) -> np.ndarray:
        """Cost column c (length R, float64, rounded to the storage precision)."""
        if self.cost is not None:
            return self.cost[c].copy()
        d = np.zeros(self.R)
        for k in range(self.xi.shape[1]):
            d += (self.xi[:, k] - self.zeta[c, k]) ** 2
        return _round(d, self.dtype)

    def q_block(self, m: int) -> np.ndarray:
        off = self.offsets
        return self.q[off[m]:off[m + 1]].copy()

    def entries(self) -> int:
        """Plan entries R*T advanced by one iteration."""
        return self.R * self.T

    def distinct_cost_columns(self) -> int:
        if self.col_index is None:
            return int(max(self.S))
        return int(np.unique(self.col_index).size)


def _round(x: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return x.astype(np.float32).astype(np.float64)
    if dtype == "f64":
        return np.asarray(x, dtype=np.float64)
    raise ValueError(f"unknown dtype {dtype!r}")


def grid_points(K: int) -> np.ndarray:
    """Pixel centres ((i+1/2)/K, (j+1/2)/K) of a K x K grid, index r = i*K + j."""
    i, j = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
    return np.stack([(i.ravel() + 0.5) / K, (j.ravel() + 0.5) / K], axis=1)


def sq_euclid(xi: np.ndarray, zeta: np.ndarray) -> np.ndarray:
    """||xi_r - zeta_s||^2 as an R x S float64 matrix."""
    d = xi[:, None, :] - zeta[None, :, :]
    return np.einsum("rsk,rsk->rs", d, d)


def grid_cost(K: int) -> np.ndarray:
    """Squared Euclidean cost between all pixels of a K x K grid, max scaled to 1."""
    pts = grid_points(K)
    c = sq_euclid(pts, pts)
    return c / c.max()


def blob_density(rng: np.random.Generator, pts: np.ndarray) -> np.ndarray:
    """Mixture of 1-3 isotropic Gaussian blobs evaluated at ``pts`` (float64).

    Centres uniform in [0.2, 0.8]^2, sigma uniform in [0.05, 0.2], mixture
    weights Dirichlet(1, ..., 1).
    """
    nb = int(rng.integers(1, 4))
    mu = rng.uniform(0.2, 0.8, size=(nb, 2))
    sig = rng.uniform(0.05, 0.2, size=nb)
    wts = rng.dirichlet(np.ones(nb))
    h = np.zeros(pts.shape[0])
    for b in range(nb):
        d2 = ((pts - mu[b]) ** 2).sum(axis=1)
        h += wts[b] / (2.0 * np.pi * sig[b] ** 2) * np.exp(-d2 / (2.0 * sig[b] ** 2))
    return h


def balanced_plain(seed: int = 0, K: int = 16, M: int = 4, iters: int = 200,
                   rho: float = 1.0, dtype: str = "f64") -> Problem:
    """Balanced WB, every measure dense on the barycenter's K x K grid.

    Default: R = S^m = 256, M = 4, FP64, 200 iterations, rho = 1.
    """
    pts = grid_points(K)
    R = K * K
    qs = []
    for m in range(M):
        rng = np.random.default_rng([1, seed, m])
        h = blob_density(rng, pts)
        qs.append(h / h.sum())
    cost = grid_cost(K)                     # symmetric: row k = column k
    return Problem(
        name=f"balanced_plain_K{K}_M{M}", R=R, S=[R] * M,
        cost=_round(cost, dtype), q=_round(np.concatenate(qs), dtype),
        col_index=None, rho=rho, gamma=float("inf"), iters=iters, dtype=dtype,
        meta={"K": K, "seed": seed})


def balanced_sparse(seed: int = 0, K: int = 64, M: int = 32, iters: int = 500,
                    rho: float = 1.0, dtype: str = "f32",
                    density_floor: float = 1e-3) -> Problem:
    """Balanced WB with sparse image-like supports (zero pixels removed).

    Each measure keeps the pixels where the raw mixture density exceeds
    ``density_floor``; its weights are the density there, normalised to sum 1.
    The barycenter lives on the full K x K grid; plan column (m, s) uses the
    grid cost column of its pixel (indexed cost).
    """
    pts = grid_points(K)
    R = K * K
    S, qs, idx = [], [], []
    for m in range(M):
        rng = np.random.default_rng([2, seed, m])
        h = blob_density(rng, pts)
        sup = np.nonzero(h > density_floor)[0]
        w = h[sup]
        S.append(int(sup.size))
        qs.append(w / w.sum())
        idx.append(sup.astype(np.int32))
    cost = grid_cost(K)
    return Problem(
        name=f"balanced_sparse_K{K}_M{M}", R=R, S=S,
        cost=_round(cost, dtype), q=_round(np.concatenate(qs), dtype),
        col_index=np.concatenate(idx).astype(np.int32), rho=rho,
        gamma=float("inf"), iters=iters, dtype=dtype,
        meta={"K": K, "seed": seed, "density_floor": density_floor})


def unbalanced_dense(seed: int = 0, K: int = 32, M: int = 50, iters: int = 1000,
                     rho: float = 1.0, gamma: float = 0.01,
                     dtype: str = "f32") -> Problem:
    """Unbalanced WB: dense blob measures with total masses uniform in [0.5, 1.5]."""
    pts = grid_points(K)
    R = K * K
    qs = []
    for m in range(M):
        rng = np.random.default_rng([3, seed, m])
        h = blob_density(rng, pts)
        mass = rng.uniform(0.5, 1.5)
        qs.append(mass * h / h.sum())
    return Problem(
        name=f"unbalanced_dense_K{K}_M{M}", R=R, S=[R] * M,
        cost=_round(grid_cost(K), dtype), q=_round(np.concatenate(qs), dtype),
        col_index=None, rho=rho, gamma=gamma, iters=iters, dtype=dtype,
        meta={"K": K, "seed": seed})


def adjoint_problem(seed: int = 0, K: int = 64, M: int = 8, iters: int = 100,
                    rho: float = 1.0, dtype: str = "f32"):
    """Dense balanced problem plus a seeded target histogram for a barycenter loss."""
    pts = grid_points(K)
    R = K * K
    qs = []
    for m in range(M):
        rng = np.random.default_rng([5, seed, m])
        h = blob_density(rng, pts)
        qs.append(h / h.sum())
    rng = np.random.default_rng([5, 999])
    tgt = blob_density(rng, pts)
    prob = Problem(
        name=f"adjoint_K{K}_M{M}", R=R, S=[R] * M,
        cost=_round(grid_cost(K), dtype), q=_round(np.concatenate(qs), dtype),
        col_index=None, rho=rho, gamma=float("inf"), iters=iters, dtype=dtype,
        meta={"K": K, "seed": seed})
    return prob, tgt / tgt.sum()


def batched_problems(n: int = 256, seed: int = 0, iters: int = 300,
                     k_range=(8, 32), m_range=(2, 8), dtype: str = "f32",
                     rho: float = 1.0) -> List[Problem]:
    """Independent balanced problems of uneven size: R = S^m = k^2, k and M uniform."""
    out = []
    rng0 = np.random.default_rng([4, seed])
    for i in range(n):
        k = int(rng0.integers(k_range[0], k_range[1] + 1))
        M = int(rng0.integers(m_range[0], m_range[1] + 1))
        pts = grid_points(k)
        qs = []
        for m in range(M):
            rng = np.random.default_rng([4, seed, i, m])
            h = blob_density(rng, pts)
            qs.append(h / h.sum())
        out.append(Problem(
            name=f"batch{i}_K{k}_M{M}", R=k * k, S=[k * k] * M,
            cost=_round(grid_cost(k), dtype), q=_round(np.concatenate(qs), dtype),
            col_index=None, rho=rho, gamma=float("inf"), iters=iters,
            dtype=dtype, meta={"K": k, "index": i}))
    return out


def tiny_problem(seed: int, R: int, S: List[int], dtype: str = "f64",
                 masses: Optional[List[float]] = None, rho: float = 1.0,
                 gamma: float = float("inf"), iters: int = 10,
                 zero_frac: float = 0.0, shared: bool = False) -> Problem:
    """Random small instance with per-column costs (or a shared cost).

    Barycenter support: R random points in [0,1]^2; measure m: S^m random
    points.  Cost = squared distance scaled to max 1.  Weights uniform in
    (0, 1] with an optional fraction of exact zeros, scaled to ``masses[m]``
    (default 1).
    """
    rng = np.random.default_rng([7, seed])
    xi = rng.uniform(0, 1, size=(R, 2))
    M = len(S)
    if shared:
        if len(set(S)) != 1:
            raise ValueError("a shared cost needs equal S^m")
        zeta = rng.uniform(0, 1, size=(S[0], 2))
        c = sq_euclid(xi, zeta)
        cost = (c / c.max()).T
        col_index = None
    else:
        blocks = []
        for m in range(M):
            zeta = rng.uniform(0, 1, size=(S[m], 2))
            blocks.append(sq_euclid(xi, zeta))
        c = np.concatenate(blocks, axis=1)
        cost = (c / c.max()).T
        col_index = np.arange(sum(S), dtype=np.int32)
    qs = []
    for m in range(M):
        w = rng.uniform(0, 1, size=S[m])
        if zero_frac > 0:
            w[rng.uniform(0, 1, size=S[m]) < zero_frac] = 0.0
            if w.sum() == 0:
                w[0] = 1.0
        mass = 1.0 if masses is None else masses[m]
        qs.append(mass * w / w.sum())
    return Problem(
        name=f"tiny_R{R}_M{M}", R=R, S=list(S), cost=_round(np.ascontiguousarray(cost), dtype),
        q=_round(np.concatenate(qs), dtype), col_index=col_index, rho=rho,
        gamma=gamma, iters=iters, dtype=dtype, meta={"seed": seed})


def line_problem(seed: int, R: int, M: int, dtype: str = "f64", rho: float = 1.0,
                 gamma: float = float("inf"), iters: int = 10) -> Problem:
    """M measures on the barycenter's own support, R points 0, 1, ..., R-1 on
    a line, with the unscaled cost c_rs = (r - s)^2 (zero diagonal, gaps of
    at least 1 off it) shared by every measure.  Weights uniform in (0, 1],
    normalised to mass 1."""
    rng = np.random.default_rng([8, seed])
    x = np.arange(R, dtype=np.float64)
    cost = (x[:, None] - x[None, :]) ** 2
    qs = []
    for _ in range(M):
        w = rng.uniform(0, 1, size=R) + 1e-3
        qs.append(w / w.sum())
    return Problem(
        name=f"line_R{R}_M{M}", R=R, S=[R] * M, cost=_round(cost, dtype),
        q=_round(np.concatenate(qs), dtype), col_index=None, rho=rho, gamma=gamma,
        iters=iters, dtype=dtype, meta={"seed": seed})


def free_support_axis(K: int, M: int):
    """(n, origin, spacing) of one axis of Xi: the averages (I + M/2)/(M K),
    I = 0, ..., M(K-1), of M pixel centres (i + 1/2)/K."""
    return M * (K - 1) + 1, (M / 2) / (M * K), 1.0 / (M * K)


def free_support_grid(K: int, M: int, d: int = 2) -> np.ndarray:
    """The set Xi of Theorem c: every average (1/M) sum_m zeta_m of M pixel
    centres ((i + 1/2)/K per axis) of a K^d grid, a uniform grid of
    ((K-1)M+1)^d points (row-major, last axis fastest).  A coordinate is
    evaluated as origin + I * spacing (one product, one sum, each rounded)."""
    n, o, h = free_support_axis(K, M)
    v = o + np.arange(n, dtype=np.float64) * h
    mesh = np.meshgrid(*([v] * d), indexing="ij")
    return np.stack([g.ravel() for g in mesh], axis=1)


def nested_ellipses(rng: np.random.Generator, K: int) -> np.ndarray:
    """A K x K image of two or three concentric, equally rotated elliptic
    rings (random centre, axes and angle), as a float64 histogram of mass 1
    on the pixel centres (row-major)."""
    c = (np.arange(K) + 0.5) / K
    X, Y = np.meshgrid(c, c, indexing="ij")
    cx, cy = rng.uniform(0.35, 0.65, size=2)
    a, b = rng.uniform(0.15, 0.3, size=2)
    phi = rng.uniform(0, np.pi)
    u = (X - cx) * np.cos(phi) + (Y - cy) * np.sin(phi)
    v = -(X - cx) * np.sin(phi) + (Y - cy) * np.cos(phi)
    rad = np.sqrt((u / a) ** 2 + (v / b) ** 2)  # 1 on the outer ellipse
    nrings = int(rng.integers(2, 4))
    scales = np.linspace(1.0, 0.3, nrings)
    width = 1.5 / (K * min(a, b))             # about 1.5 pixels, in units of rad
    h = sum(np.exp(-((rad - sc) ** 2) / (2 * width ** 2)) for sc in scales).ravel()
    return h / h.sum()


def free_support(seed: int = 0, K: int = 60, M: int = 10, dtype: str = "f32", rho: float = 1.0,
                 iters: int = 100) -> Problem:
    """Free-support barycenter of M nested-ellipse images on a K x K grid with
    alpha_m = 1/M (Theorem c): support Xi of ((K-1)M+1)^2 points (349,281 for
    K = 60, M = 10), S^m = K^2 pixels per measure (all kept; weights that
    round to zero project to zero columns), squared Euclidean cost between
    Xi and the pixel centres, not scaled.  The cost is given by its points
    (xi, zeta): it is R x K^2 values per measure-independent column set."""
    rng = np.random.default_rng([9, seed])
    xi = free_support_grid(K, M)
    c = (np.arange(K) + 0.5) / K
    X, Y = np.meshgrid(c, c, indexing="ij")
    zeta = np.stack([X.ravel(), Y.ravel()], axis=1)
    q = np.concatenate([nested_ellipses(rng, K) for _ in range(M)])
    S = K * K
    n, o, h = free_support_axis(K, M)
    return Problem(
        name=f"free_support_K{K}_M{M}", R=xi.shape[0], S=[S] * M, cost=None, q=_round(q, dtype),
        col_index=None, rho=rho, iters=iters, dtype=dtype,
        meta={"K": K, "M": M, "seed": seed, "grid": ([n, n], [o, o], [h, h])}, xi=xi, zeta=zeta)


def bundle_sequence(bundles, iters: int, seed: int = 0, alpha=None) -> np.ndarray:
    """Seeded draws for the randomized variant: iteration k takes bundle i
    with probability beta_i = sum of alpha_m over the bundle's measures
    (alpha uniform by default).  Returns ``iters`` bundle indices (int32)."""
    M = sum(len(b) for b in bundles)
    a = np.full(M, 1.0 / M) if alpha is None else np.asarray(alpha, dtype=np.float64)
    beta = np.array([a[list(b)].sum() for b in bundles])
    rng = np.random.default_rng([6, seed])
    return rng.choice(len(bundles), size=iters, p=beta / beta.sum()).astype(np.int32)
