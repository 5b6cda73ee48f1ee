"""Parity at full size, in the benchmark's launch configuration: the
balanced sparse workload (64x64 grid, 32 measures, T = 97,894 columns) with
the default schedule.  The oracle cannot run whole iterations at this size
in a test, but one iteration's columns are independent given the marginals
(Alg. 1 Step 2), so sampled columns of theta^{k+1} are recomputed by the
oracle from the GPU's theta^k and marginals; the marginals are checked
against a plain FP64 sum of theta^k (within the storage rounding), and the
mass invariant over all columns."""
import sys

import numpy as np
import pytest
import torch

from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_marginals_of_stored(pm, th, off, dtype):
    """The device's marginals p^(m) are FP64 row sums of the updates before
    they are rounded to the storage type (the rounding of the inactive
    entries' common value -b would otherwise add up over the S^m columns of
    a measure).  Every stored entry is its update rounded to nearest, so in
    FP32 each row sum of the stored plans lies within 2^-24 sum_s |theta_rs|
    of p^(m)_r (plus FP64 summation noise); in FP64 the two agree to 1e-12."""
    M = len(off) - 1
    st = np.stack([th[off[m]:off[m + 1]].sum(axis=0, dtype=np.float64) for m in range(M)])
    if dtype == "f64":
        e = np.abs(pm - st).max() / np.abs(st).max()
        say(f"marginals vs FP64 sums of the stored plans: max rel {e:.2e}")
        assert e <= 1e-12
        return
    ab = np.stack([np.abs(th[off[m]:off[m + 1]]).sum(axis=0, dtype=np.float64) for m in range(M)])
    err = np.abs(pm - st)
    say(f"marginals vs FP64 sums of the stored FP32 plans: max |diff| / rounding bound "
        f"{np.max(err / np.maximum(2.0 ** -24 * ab, 1e-300)):.3f}")
    assert np.all(err <= 2.0 ** -24 * ab * (1 + 1e-6) + 1e-12 * np.abs(st).max())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_balanced_sparse_full_size_sampled_columns(dtype):
    p = inputs.balanced_sparse(dtype=dtype)
    say(f"{p.name} {dtype}: R={p.R} M={p.M} T={p.T}")
    s = mam.solver_for(p)
    say(f"schedule {s.schedule()}")
    s.init()
    s.iterate(5)
    torch.cuda.synchronize()
    th5 = s.theta[:, :p.R].cpu().numpy()              # theta^5, row j = plan column j
    pm = s.marginals().cpu().numpy()
    off = p.offsets
    check_marginals_of_stored(pm, th5, off, dtype)
    s.iterate(1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1234)
    cols = np.sort(np.concatenate([rng.choice(np.arange(off[m], off[m + 1]), size=3, replace=False)
                                   for m in range(p.M)]))
    meas = np.searchsorted(off, cols, side="right") - 1
    new, _, t = O.mam_step_columns(th5[cols].T.astype(np.float64), meas, pm,
                                   p.cost[p.col_index[cols]].T.astype(np.float64),
                                   p.q[cols].astype(np.float64), p.S, p.rho, p.gamma)
    got = s.theta[torch.as_tensor(cols, device=s.theta.device), :p.R].double().cpu().numpy().T
    # FP32: the GPU rounds theta' once to float after FP64 arithmetic, so each
    # entry is within 2 float ulps.  FP64: the inactive entries are -b =
    # -(p - p^(m))/S^m, a difference of nearly equal marginals whose summation
    # order differs, so entries are compared relative to the column's largest.
    err = np.abs(got - new)
    if dtype == "f32":
        rel_e = np.max(err / np.maximum(np.abs(new), 1e-300))
        say(f"{len(cols)} sampled columns: max |diff| / |value| = {rel_e:.2e}")
        assert np.all(err <= 2.0 ** -23 * np.abs(new))
    else:
        rel_c = np.max(err.max(axis=0) / np.abs(new).max(axis=0))
        say(f"{len(cols)} sampled columns: max over columns of ||diff||_inf / ||column||_inf = {rel_c:.2e}")
        assert rel_c <= 1e-12
    # mass invariant over every column of theta^6: each p^(m) keeps the mass 1
    pm6 = s.marginals().cpu().numpy()
    drift = np.abs(pm6.sum(axis=1) - 1.0).max()
    say(f"mass drift after 6 iterations: {drift:.2e}")
    assert drift <= (1e-5 if dtype == "f32" else 1e-12)


def test_unbalanced_full_size_sampled_columns():
    """32x32 grid, 50 dense measures with masses in [0.5, 1.5], gamma = 0.01,
    FP32, default schedule: theta^6 columns from the GPU's theta^5 through
    the oracle's step (including the damping t^k < 1)."""
    p = inputs.unbalanced_dense()
    say(f"{p.name}: R={p.R} M={p.M} T={p.T} gamma={p.gamma}")
    s = mam.solver_for(p)
    say(f"schedule {s.schedule()}")
    s.init()
    s.iterate(5)
    torch.cuda.synchronize()
    th5 = s.theta[:, :p.R].cpu().numpy()
    off = p.offsets
    pm = s.marginals().cpu().numpy()
    check_marginals_of_stored(pm, th5, off, "f32")
    s.iterate(1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    cols = np.sort(np.concatenate([rng.choice(np.arange(off[m], off[m + 1]), size=2, replace=False)
                                   for m in range(p.M)]))
    meas = np.searchsorted(off, cols, side="right") - 1
    cost_cols = np.stack([p.cost[c - off[m]] for c, m in zip(cols, meas)], axis=1).astype(np.float64)
    new, _, t = O.mam_step_columns(th5[cols].T.astype(np.float64), meas, pm, cost_cols,
                                   p.q[cols].astype(np.float64), p.S, p.rho, p.gamma)
    got = s.theta[torch.as_tensor(cols, device=s.theta.device), :p.R].double().cpu().numpy().T
    err = np.abs(got - new)
    say(f"t^5 = {t:.6f}; {len(cols)} sampled columns: max |diff| / |value| = "
        f"{np.max(err / np.maximum(np.abs(new), 1e-300)):.2e}")
    assert t < 1.0
    assert np.all(err <= 2.0 ** -23 * np.abs(new))


def test_batch_of_256_full_size_sampled_problems():
    """All 256 problems of the batched workload with the benchmark's launch
    configuration (autotuned schedules, graph replay); four problems (the
    smallest, the largest and two drawn at random) against the oracle."""
    from paper_2309_05315_amd import autotune
    probs = inputs.batched_problems(iters=12)
    scheds = autotune.tune_batch(probs, use_cache=False)
    b = mam.Batch(probs, schedules=scheds)
    b.graph(6)
    b.init()
    b.iterate(12)
    torch.cuda.synchronize()
    sizes = [p.R * p.T for p in probs]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))} |
                  set(np.random.default_rng(7).choice(len(probs), 2, replace=False).tolist()))
    for i in pick:
        p = probs[i]
        ref = O.mam([p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)],
                    p.rho, p.gamma, 12)["p_bar"]
        got = b.barycenter(i).cpu().numpy()
        e = np.abs(got - ref).sum() / np.abs(ref).sum()
        say(f"problem {i} {p.name}: rel L1 {e:.2e}")
        assert e <= 1e-5


@pytest.mark.parametrize("grid,sparse", [(False, False), (True, False), (True, True)])
def test_free_support_full_size_sampled_columns(grid, sparse):
    """Free-support barycenter of 10 nested-ellipse 60x60 images: the R =
    349,281 support points of Theorem c, T = 36,000 columns, 50 GB of FP32
    plans, default long-column schedule.  theta^6 columns from the GPU's
    theta^5 through the oracle's step with the oracle's own cost (built from
    the points in FP64 and rounded once to float, as the device builds it;
    the two may differ by one float ulp, and the projection moves at most
    twice as far as w, which the tolerance allows; with grid = True the
    kernels form the cost from the grid in the oracle's operation order, so
    the two costs are the same).  The marginal of measure 0 is checked
    against a plain FP64 sum of its 3,600 columns.  With the sparse store the
    plans live as -b plus patches between the iterations of each call and are
    written back when it returns."""
    p = inputs.free_support(dtype="f32")
    say(f"{p.name}: R={p.R} M={p.M} T={p.T} grid cost {grid} sparse store {sparse}")
    s = mam.solver_for(p, grid=grid, sparse_store=sparse)
    sc = s.schedule()
    say(f"schedule {sc}")
    assert sc["rows_per_tile"] > 0
    s.init()
    s.iterate(5)
    torch.cuda.synchronize()
    off = p.offsets
    rng = np.random.default_rng(4321)
    cols = np.sort(np.concatenate([rng.choice(np.arange(off[m], off[m + 1]), size=3, replace=False)
                                   for m in range(p.M)]))
    cols_t = torch.as_tensor(cols, device=s.theta.device)
    th5 = s.theta[cols_t, :p.R].double().cpu().numpy()
    pm5 = s.marginals().cpu().numpy()
    pm0, ab0 = np.zeros(p.R), np.zeros(p.R)
    for c0 in range(off[0], off[1], 360):
        blk = s.theta[c0:min(c0 + 360, off[1]), :p.R].cpu().numpy().astype(np.float64)
        pm0 += blk.sum(axis=0)
        ab0 += np.abs(blk).sum(axis=0)
    e_pm = np.abs(pm5[0] - pm0)
    say(f"marginal of measure 0 over theta^5: max |diff| / rounding bound "
        f"{np.max(e_pm / np.maximum(2.0 ** -24 * ab0, 1e-300)):.3f}")
    assert np.all(e_pm <= 2.0 ** -24 * ab0 * (1 + 1e-6) + 1e-12 * np.abs(pm0).max())
    s.iterate(1)
    torch.cuda.synchronize()
    meas = np.searchsorted(off, cols, side="right") - 1
    cost_cols = np.stack([p.cost_column(int(c - off[m])) for c, m in zip(cols, meas)], axis=1)
    new, _, t = O.mam_step_columns(th5.T, meas, pm5, cost_cols, p.q[cols].astype(np.float64), p.S, p.rho,
                                   p.gamma)
    got = s.theta[cols_t, :p.R].double().cpu().numpy().T
    if grid:
        dc = np.zeros(len(cols))
    else:
        dc = np.abs(s.cost[torch.as_tensor(cols - off[meas], device=s.cost.device), :p.R].double().cpu().numpy().T
                    - cost_cols).max(axis=0)
        say(f"device cost vs oracle cost on the sampled columns: max |diff| {dc.max():.2e}")
        assert np.all(dc <= 2.0 ** -23 * np.abs(cost_cols).max(axis=0))
    err = np.abs(got - new)
    bound = 2.0 ** -23 * np.abs(new) + 2.0 * dc[None, :] / p.rho
    say(f"{len(cols)} sampled columns: max |diff| / bound = {np.max(err / np.maximum(bound, 1e-300)):.3f}")
    assert np.all(err <= bound)
    drift = np.abs(s.marginals().cpu().numpy().sum(axis=1) - 1.0).max()
    say(f"mass drift after 6 iterations: {drift:.2e}")
    assert drift <= 1e-5
