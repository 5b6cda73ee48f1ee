"""Sub-wave column groups (16 or 32 lanes per column, several columns per
wave) against the FP64 oracle, element by element (MI355X only).

Same tolerances as the one-wave kernel: 1e-10 (FP64 plans) and 1e-5 (FP32
plans) relative on the barycenter, every plan entry and the marginals.
Cases span: a column shorter than the group, one value per lane, ragged last
vectors, every cost layout, zero weights (columns that stay 0), unbalanced
damping, relaxed measure constraints, cold starts, batches of uneven
problems with graph replay, and the randomized variant.
"""
import dataclasses
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


def blocks(p):
    return [p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)]


def rel(a, b, ord=1):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    if ord == 1:
        return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check(p, iters, relaxed=False, **sched):
    cost, q = blocks(p)
    ora = O.mam(cost, q, p.rho, p.gamma, iters, relaxed=relaxed)
    s = mam.solver_for(p, relaxed=relaxed, **sched)
    sc = s.schedule()
    assert sc["threads_per_column"] == sched["threads_per_column"], sc
    s.init()
    s.iterate(iters)
    tol = TOL[p.dtype]
    pb = s.barycenter().cpu().numpy()
    e1, einf = rel(pb, ora["p_bar"]), rel(pb, ora["p_bar"], np.inf)
    eth = max(rel(a, b, np.inf) for a, b in zip(s.plans(), ora["theta"]))
    epm = np.abs(s.marginals().cpu().numpy() - ora["pm"]).max() / np.abs(ora["pm"]).max()
    say(f"{p.name} {p.dtype} R={p.R} S={p.S[:4]} sched={sc}: p_bar rel L1 {e1:.2e} max {einf:.2e}, "
        f"plans {eth:.2e}, marginals {epm:.2e}")
    assert e1 <= tol and einf <= tol and eth <= tol and epm <= tol
    return s


CASES = [
    # (name, builder, lanes)
    ("R=7, shorter than a group", lambda dt: inputs.tiny_problem(1, R=7, S=[5, 6, 4], dtype=dt, zero_frac=0.2), 16),
    ("R=16, one value per lane", lambda dt: inputs.tiny_problem(2, R=16, S=[9, 11], dtype=dt), 16),
    ("R=64, shared cost", lambda dt: inputs.tiny_problem(3, R=64, S=[64, 64], dtype=dt, shared=True), 16),
    ("R=100, ragged vectors", lambda dt: inputs.tiny_problem(4, R=100, S=[30, 41, 7], dtype=dt), 16),
    ("R=121, 32 lanes", lambda dt: inputs.tiny_problem(5, R=121, S=[33, 28], dtype=dt), 32),
    ("R=256, 16 values per lane", lambda dt: inputs.tiny_problem(6, R=256, S=[20, 13], dtype=dt), 16),
    ("R=500, 32 lanes, 16 values", lambda dt: inputs.tiny_problem(7, R=500, S=[17, 9], dtype=dt), 32),
    ("grid K=8, indexed sparse", lambda dt: inputs.balanced_sparse(K=8, M=5, dtype=dt), 16),
    ("unbalanced damping", lambda dt: inputs.tiny_problem(8, R=90, S=[30, 22, 15], masses=[0.6, 1.0, 1.5],
                                                          gamma=0.02, dtype=dt), 32),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_subwave_matches_oracle(case, dtype):
    name, build, lanes = CASES[case]
    say(f"case {name}, {lanes} lanes per column")
    check(build(dtype), 20, threads_per_column=lanes)


@pytest.mark.parametrize("lanes", [16, 32])
def test_subwave_cold_start_and_many_workgroups(lanes):
    p = inputs.tiny_problem(9, R=60, S=[50, 70, 33], dtype="f64", zero_frac=0.3)
    check(p, 15, threads_per_column=lanes, cold=True)
    check(p, 15, threads_per_column=lanes, workgroups=1)
    check(p, 15, threads_per_column=lanes, workgroups=500)


@pytest.mark.parametrize("eta,gamma", [(0.002, 0.2), (0.02, math.inf)])
def test_subwave_relaxed_constraints(eta, gamma):
    # distances d = c - eta of the extension (the cases where part of a
    # column's mass stays unassigned)
    p = inputs.tiny_problem(31, R=150, S=[40, 25, 33], dtype="f64", masses=[0.7, 1.0, 1.3], gamma=gamma)
    p = dataclasses.replace(p, cost=p.cost - eta)
    check(p, 40, relaxed=True, threads_per_column=16)


def test_subwave_bitwise_reproducible_and_graph_equals_eager():
    p = inputs.tiny_problem(11, R=200, S=[60, 45, 31], dtype="f32")
    out = []
    for graph in (0, 0, 5):
        s = mam.solver_for(p, threads_per_column=16)
        if graph:
            s.graph(graph)
        s.init()
        s.iterate(20)
        out.append((s.barycenter().cpu().numpy(), s.plans()))
        s.close()
    for pb, th in out[1:]:
        assert np.array_equal(pb, out[0][0])
        for a, b in zip(th, out[0][1]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_with_subwave_groups(dtype):
    """Uneven small problems in one batch, each shape group on 16 or 32 lanes
    per column, replayed from a graph."""
    probs = [inputs.tiny_problem(20 + i, R=R, S=S, dtype=dtype)
             for i, (R, S) in enumerate([(49, [40, 23]), (64, [64, 10, 5]), (81, [17, 60]),
                                         (121, [30, 30, 30]), (144, [12, 9]), (256, [40, 7])])]
    probe = mam.Batch(probs)
    groups = probe.groups()
    probe.close()
    scheds = {g: {"threads_per_column": 16 if g % 2 == 0 else 32} for g in range(groups)}
    b = mam.Batch(probs, schedules=scheds)
    say(f"batch: {[b.schedule(g) for g in range(b.groups())]}")
    b.graph(5)
    b.init()
    b.iterate(20)
    for i, p in enumerate(probs):
        cost, q = blocks(p)
        ref = O.mam(cost, q, p.rho, p.gamma, 20)["p_bar"]
        e = rel(b.barycenter(i).cpu().numpy(), ref)
        say(f"  problem {i} R={p.R} group {b.group_of(i)}: rel L1 {e:.2e}")
        assert e <= TOL[dtype]
    b.close()


def test_randomized_with_subwave_groups():
    p = inputs.tiny_problem(30, R=130, S=[40, 25, 60, 33], dtype="f64")
    bundles = [[0, 2], [1], [3]]
    bundle_of = [0, 1, 0, 2]
    seq = inputs.bundle_sequence(bundles, 30, seed=3)
    ora = O.mam([p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)], p.rho, p.gamma,
                30, bundles=bundles, seq=seq)
    s = mam.solver_for(p, threads_per_column=32)
    s.init()
    s.set_bundles(bundle_of)
    s.iterate_bundles(seq)
    assert rel(s.barycenter().cpu().numpy(), ora["p_bar"]) <= 1e-10


def test_subwave_rejects_diagnostics_and_reverse_mode():
    p = inputs.tiny_problem(12, R=50, S=[10, 12], dtype="f64")
    s = mam.solver_for(p, threads_per_column=16, diag=True)
    s.init()
    with pytest.raises(mam.MAMError):
        s.iterate(2)
    s = mam.solver_for(p, threads_per_column=16)
    s.init()
    with pytest.raises(mam.MAMError):
        s.record(3)
    with pytest.raises(mam.MAMError):
        mam.solver_for(p, threads_per_column=16, columns_in_flight=2)
    with pytest.raises(mam.MAMError):
        mam.solver_for(inputs.tiny_problem(13, R=300, S=[5], dtype="f64"), threads_per_column=16)
