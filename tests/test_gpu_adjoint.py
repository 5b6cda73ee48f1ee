"""Reverse mode on the GPU: gradients of a barycenter loss with respect to
q and the cost, against the FP64 gradient oracle (torch autograd through a
CPU re-implementation of the iteration) and central finite differences."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mam_grad as G
from oracle import mam_oracle as O
from paper_2309_05315_amd import inputs
from paper_2309_05315_amd import mam
from paper_2309_05315_amd.autograd import barycenter

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def fold_cost(p, gblocks):
    """Per-measure R x S^m cost gradients summed into the cost's storage (ncols x R)."""
    out = np.zeros(p.cost.shape, dtype=np.float64)
    for m in range(p.M):
        np.add.at(out, p.cost_columns(m), gblocks[m].T)
    return out


def indexed_tiny(seed, R, S, dtype="f64", ncols=9):
    base = inputs.tiny_problem(seed, R=R, S=[ncols], dtype=dtype, shared=True)
    rng = np.random.default_rng([11, seed])
    idx = np.sort(rng.integers(0, ncols, size=sum(S))).astype(np.int32)
    q = np.concatenate([inputs.tiny_problem(seed + 100, R=R, S=[s], dtype=dtype).q for s in S])
    return inputs.Problem(name=f"indexed_R{R}", R=R, S=list(S), cost=base.cost, q=q, col_index=idx,
                          rho=1.0, gamma=math.inf, iters=10, dtype=dtype, meta={})


def gpu_grads(p, iters, grad_p=None, target=None, ckpt_every=0, **sched):
    s = mam.solver_for(p, **sched)
    s.init()
    s.record(iters, ckpt_every)
    pbar = s.barycenter()
    if grad_p is None:
        grad_p = 2.0 * (pbar - torch.as_tensor(target, device=pbar.device))
    gq, gc = s.backward(torch.as_tensor(grad_p, dtype=torch.float64))
    torch.cuda.synchronize()
    return (pbar.cpu().numpy(), gq.double().cpu().numpy(), gc[:, :p.R].double().cpu().numpy(), s)


CASES = {
    "percol_R7": lambda dt: inputs.tiny_problem(1, R=7, S=[5, 6, 4], dtype=dt, zero_frac=0.2),
    "shared_R64": lambda dt: inputs.tiny_problem(2, R=64, S=[64, 64], dtype=dt, shared=True),
    "percol_R65": lambda dt: inputs.tiny_problem(3, R=65, S=[30, 41], dtype=dt),
    "percol_R200": lambda dt: inputs.tiny_problem(4, R=200, S=[17, 60, 5], dtype=dt),
    "percol_R600": lambda dt: inputs.tiny_problem(16, R=600, S=[11, 7], dtype=dt),
    "percol_R1030": lambda dt: inputs.tiny_problem(5, R=1030, S=[12, 9], dtype=dt),
    "percol_R4099": lambda dt: inputs.tiny_problem(6, R=4099, S=[6, 7], dtype=dt),
    "indexed_R50": lambda dt: indexed_tiny(7, R=50, S=[20, 13], dtype=dt),
    "grid_K8_M3": lambda dt: inputs.balanced_plain(K=8, M=3, dtype=dt),
    # the reverse kernel finds a column's measure by one ballot up to 65
    # measures and by a search beyond
    "percol_M65": lambda dt: inputs.tiny_problem(13, R=24, S=[3, 1, 2, 4] * 16 + [2], dtype=dt),
    "percol_M66": lambda dt: inputs.tiny_problem(14, R=24, S=[3, 1, 2, 4] * 16 + [2, 5], dtype=dt),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradients_match_oracle(name, dtype):
    p = CASES[name](dtype)
    iters = 12
    tgt = np.random.default_rng(5).dirichlet(np.ones(p.R))
    cost, q = blocks(p)
    L, pbar_o, gq_o, gc_o = G.loss_and_grads(cost, q, p.rho, iters, tgt)
    pbar, gq, gc, s = gpu_grads(p, iters, target=tgt)
    gq_o = np.concatenate(gq_o)
    gc_o = fold_cost(p, gc_o)
    eq, ec = rel(gq, gq_o), rel(gc, gc_o)
    say(f"{name} {dtype} sched={s.schedule()} rel L1: q {eq:.2e}, cost {ec:.2e}")
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert eq <= tol and ec <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vector_jacobian_product_matches_oracle(dtype):
    p = inputs.tiny_problem(9, R=40, S=[25, 31, 18], dtype=dtype)
    u = np.random.default_rng(9).normal(size=p.R)
    cost, q = blocks(p)
    _, gq_o, gc_o = G.vjp(cost, q, p.rho, 15, u)
    _, gq, gc, _ = gpu_grads(p, 15, grad_p=u)
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert rel(gq, np.concatenate(gq_o)) <= tol
    assert rel(gc, fold_cost(p, gc_o)) <= tol


def test_checkpoint_windows_and_repeated_backward_are_bitwise_equal():
    p = inputs.tiny_problem(10, R=300, S=[40, 33], dtype="f32")
    u = np.random.default_rng(10).normal(size=p.R)
    ref = None
    for C in (0, 1, 3, 4, 10, 25):
        _, gq, gc, s = gpu_grads(p, 10, grad_p=u, ckpt_every=C)
        say(f"ckpt_every={C}: adjoint workspace {s.adj_workspace.numel()} bytes")
        if ref is None:
            ref = (gq, gc)
        assert np.array_equal(gq, ref[0]) and np.array_equal(gc, ref[1]), C
        gq2, gc2 = s.backward(torch.as_tensor(u))
        assert np.array_equal(gq2.double().cpu().numpy(), gq)
        assert np.array_equal(gc2[:, :p.R].double().cpu().numpy(), gc)


def test_zero_loss_gradient_gives_zero_gradients():
    """dL/dp_bar = 0: every adjoint is 0 (the fixed-point row sums then run
    at scale 1 and stay 0)."""
    p = inputs.tiny_problem(15, R=50, S=[20, 13], dtype="f64")
    _, gq, gc, _ = gpu_grads(p, 8, grad_p=np.zeros(p.R))
    assert np.all(gq == 0.0) and np.all(gc == 0.0)


def test_zero_iterations():
    p = inputs.tiny_problem(11, R=33, S=[7, 9])
    u = np.random.default_rng(11).normal(size=p.R)
    cost, q = blocks(p)
    _, gq_o, gc_o = G.vjp(cost, q, p.rho, 0, u)
    _, gq, gc, _ = gpu_grads(p, 0, grad_p=u)
    assert rel(gq, np.concatenate(gq_o)) <= 1e-12
    assert np.all(gc == 0.0)


def test_record_matches_plain_iteration():
    p = inputs.tiny_problem(12, R=129, S=[50, 70], dtype="f32")
    a = mam.solver_for(p)
    a.init()
    a.iterate(20)
    b = mam.solver_for(p)
    b.init()
    b.record(20, 6)
    assert np.array_equal(a.barycenter().cpu().numpy(), b.barycenter().cpu().numpy())
    for x, y in zip(a.plans(), b.plans()):
        assert np.array_equal(x, y)


def test_autograd_function_and_gradcheck():
    p = inputs.tiny_problem(13, R=6, S=[5, 4], dtype="f64")
    cost = torch.tensor(p.cost, device="cuda", requires_grad=True)
    q = torch.tensor(p.q, device="cuda", requires_grad=True)
    tgt = torch.full((p.R,), 1.0 / p.R, dtype=torch.float64, device="cuda")
    pbar = barycenter(cost, q, p.S, rho=p.rho, iters=9, cost_mode=mam.COST_PER_COLUMN)
    loss = ((pbar - tgt) ** 2).sum()
    loss.backward()
    c_np, q_np = blocks(p)
    _, _, gq_o, gc_o = G.loss_and_grads(c_np, q_np, p.rho, 9, tgt.cpu().numpy())
    assert rel(q.grad.cpu().numpy(), np.concatenate(gq_o)) <= 1e-9
    assert rel(cost.grad.cpu().numpy(), fold_cost(p, gc_o)) <= 1e-9
    # finite differences in the cost (q moves would change the masses)
    f = lambda c: barycenter(c, q.detach(), p.S, rho=p.rho, iters=9, cost_mode=mam.COST_PER_COLUMN)
    assert torch.autograd.gradcheck(f, (cost.detach().clone().requires_grad_(True),), eps=1e-7,
                                    atol=1e-6, rtol=1e-5)


def test_adjoint_problem_full_size_vs_finite_differences():
    """The 64 x 64 grid, 8 measures, 100 iterations: FP64 reverse sweep
    against central differences of the FP64 forward along mass-preserving
    relative directions in q and relative directions in c, and the FP32
    reverse sweep (windows of 10 iterations) against the FP64 one."""
    p64, tgt = inputs.adjoint_problem(dtype="f64")
    p32, _ = inputs.adjoint_problem(dtype="f32")
    iters = p64.iters
    say(f"adjoint problem R={p64.R} M={p64.M} T={p64.T} iters={iters}")
    _, gq64, gc64, _ = gpu_grads(p64, iters, target=tgt)
    _, gq32, gc32, s32 = gpu_grads(p32, iters, target=tgt, ckpt_every=10)
    say(f"FP32 vs FP64 gradients rel L1: q {rel(gq32, gq64):.2e} cost {rel(gc32, gc64):.2e}")
    assert rel(gq32, gq64) <= 1e-4 and rel(gc32, gc64) <= 1e-4

    dev = "cuda"
    s = mam.solver_for(p64)
    q0 = s.q.clone()
    c0 = s.cost.clone()
    tgt_t = torch.as_tensor(tgt, device=dev)

    def loss():
        s.init()
        s.iterate(iters)
        return float(((s.barycenter() - tgt_t) ** 2).sum())

    rng = np.random.default_rng(77)
    off = p64.offsets
    h = 1e-6
    cmax = float(c0.abs().max())
    worst = 0.0
    for trial in range(4):
        # q: q * (1 + h u) with u Rademacher, projected to keep every measure's mass
        u = rng.choice([-1.0, 1.0], size=p64.T)
        d = p64.q * u
        for m in range(p64.M):
            sl = slice(off[m], off[m + 1])
            d[sl] -= p64.q[sl] * d[sl].sum() / p64.q[sl].sum()
        dt = torch.as_tensor(d, device=dev)
        s.q.copy_(q0 + h * dt)
        lp = loss()
        s.q.copy_(q0 - h * dt)
        lm = loss()
        s.q.copy_(q0)
        fd = (lp - lm) / (2 * h)
        an = float(gq64 @ d)
        e = abs(fd - an) / max(abs(an), 1e-300)
        say(f"q direction {trial}: FD {fd:.10e} adjoint {an:.10e} rel {e:.2e}")
        worst = max(worst, e)
        # c: c + hc u max|c|.  The map is piecewise affine: a step must not
        # move any w across its column's threshold, and the cost moves w
        # directly (by hc max|c| per entry, against q_s ~ 2e-4), so hc is
        # far smaller than the relative step in q.  Two step sizes show the
        # difference quotient has settled.
        uc = torch.as_tensor(rng.choice([-1.0, 1.0], size=(p64.cost.shape[0], p64.R)), device=dev)
        an = float((gc64 * uc.cpu().numpy()).sum() * cmax)
        fds = []
        for hc in (2.5e-10, 6.25e-11):
            s.cost[:, :p64.R].copy_(c0[:, :p64.R] + hc * cmax * uc)
            lp = loss()
            s.cost[:, :p64.R].copy_(c0[:, :p64.R] - hc * cmax * uc)
            lm = loss()
            s.cost.copy_(c0)
            fds.append((lp - lm) / (2 * hc))
        e = abs(fds[1] - an) / max(abs(an), 1e-300)
        say(f"c direction {trial}: FD {fds[1]:.10e} (4x step {fds[0]:.10e}) adjoint {an:.10e} rel {e:.2e}")
        worst = max(worst, e)
    assert worst <= 1e-4


def test_reverse_mode_errors():
    p = inputs.tiny_problem(15, R=20, S=[5, 6])
    s = mam.solver_for(p)
    s.init(torch.full_like(s.theta, 0.01))
    with pytest.raises(mam.MAMError, match="MAM_ESTATE"):
        s.record(5)
    s.init()
    s.iterate(1)
    with pytest.raises(mam.MAMError, match="MAM_ESTATE"):
        s.record(5)
    s.init()
    with pytest.raises(mam.MAMError, match="MAM_ESTATE"):
        s.backward(torch.zeros(p.R, dtype=torch.float64))
    s.record(5)
    s.backward(torch.ones(p.R, dtype=torch.float64))
    with pytest.raises(mam.MAMError, match="MAM_ESTATE"):
        s.iterate(1)   # the reverse sweep leaves an intermediate iterate


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradients_large_rho(dtype):
    """Large active sets: most threads hold more than two active entries, so
    the reverse kernel's general path does the work."""
    p = inputs.balanced_plain(K=10, M=3, dtype=dtype)
    p.rho = float(p.R * np.mean(p.S))
    iters = 15
    tgt = np.random.default_rng(6).dirichlet(np.ones(p.R))
    cost, q = blocks(p)
    _, _, gq_o, gc_o = G.loss_and_grads(cost, q, p.rho, iters, tgt)
    _, gq, gc, _ = gpu_grads(p, iters, target=tgt)
    eq, ec = rel(gq, np.concatenate(gq_o)), rel(gc, fold_cost(p, gc_o))
    say(f"large rho {dtype}: rel L1 q {eq:.2e} cost {ec:.2e}")
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert eq <= tol and ec <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ckpt", [0, 4])
def test_unbalanced_gradients_match_oracle(dtype, ckpt):
    """Finite gamma with the damping active (t < 1 from the second iteration
    on): the rank-one term of the transposed averaging, against the gradient
    oracle."""
    p = inputs.tiny_problem(16, R=90, S=[30, 45, 20], dtype=dtype, masses=[0.6, 1.0, 1.5], gamma=0.02)
    iters = 12
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, iters, record=True)
    assert max(ora["hist"]["t"][1:]) < 1.0
    tgt = np.random.default_rng(8).dirichlet(np.ones(p.R))
    _, _, gq_o, gc_o = G.loss_and_grads(cost, q, p.rho, iters, tgt, p.gamma)
    _, gq, gc, _ = gpu_grads(p, iters, target=tgt, ckpt_every=ckpt)
    eq, ec = rel(gq, np.concatenate(gq_o)), rel(gc, fold_cost(p, gc_o))
    say(f"unbalanced {dtype} ckpt={ckpt}: rel L1 q {eq:.2e} cost {ec:.2e}")
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert eq <= tol and ec <= tol


def test_unbalanced_gradients_mixed_damping():
    """gamma between the damped and undamped regimes: t = 1 at some
    iterations and t < 1 at others."""
    p = inputs.tiny_problem(17, R=50, S=[20, 25], masses=[0.9, 1.1], gamma=0.2)
    iters = 15
    cost, q = blocks(p)
    ts = O.mam(cost, q, p.rho, p.gamma, iters, record=True)["hist"]["t"]
    say(f"t history: min {min(ts):.3f} max {max(ts):.3f}")
    assert min(ts) < 1.0 and max(ts) == 1.0
    u = np.random.default_rng(9).normal(size=p.R)
    _, gq_o, gc_o = G.vjp(cost, q, p.rho, iters, u, p.gamma)
    _, gq, gc, _ = gpu_grads(p, iters, grad_p=u)
    assert rel(gq, np.concatenate(gq_o)) <= 1e-9
    assert rel(gc, fold_cost(p, gc_o)) <= 1e-9
