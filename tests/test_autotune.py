"""Autotuner: candidate lists and cache keys (CPU); tuned schedules run and
keep results within tolerance of the oracle (GPU)."""
import numpy as np
import pytest

from paper_2309_05315_amd import autotune, inputs


def test_candidates_and_keys():
    p = inputs.tiny_problem(1, R=300, S=[40, 17], dtype="f32", shared=False)
    c = autotune.candidates(p)
    # float, R = 300: 64 by default, its neighbours, and sub-wave groups of 16 and 32 lanes
    assert {x["threads_per_column"] for x in c} == {16, 32, 64, 128}
    assert all(x["columns_in_flight"] == 1 for x in c if x["threads_per_column"] < 64)
    assert all(x["order"] == 0 for x in c)          # per-column cost: one order only
    q = inputs.tiny_problem(1, R=64, S=[64, 64], dtype="f32", shared=True)
    assert {x["order"] for x in autotune.candidates(q)} == {1, 2}
    assert autotune.problem_key(p) == autotune.problem_key(inputs.tiny_problem(1, R=300, S=[40, 17], dtype="f32"))
    assert autotune.problem_key(p) != autotune.problem_key(q)


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("MAM_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    assert autotune.cache_path() == str(tmp_path / "c.json")


@pytest.mark.gpu
def test_tuned_schedule_runs_and_matches_oracle(monkeypatch, tmp_path):
    import json
    from oracle import mam_oracle as O
    from paper_2309_05315_amd import mam
    monkeypatch.setenv("MAM_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    p = inputs.balanced_sparse(K=16, M=6, dtype="f32")
    sc = autotune.tune(p, iters=3, warm=1)
    assert json.load(open(tmp_path / "c.json"))          # cached
    assert autotune.tune(p) == sc                          # served from the cache
    s = mam.solver_for(p, **sc)
    s.init()
    s.iterate(10)
    ref = O.mam([p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)], p.rho, p.gamma, 10)["p_bar"]
    got = s.barycenter().cpu().numpy()
    assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-5


@pytest.mark.gpu
def test_tuned_batch_matches_oracle(monkeypatch, tmp_path):
    from oracle import mam_oracle as O
    from paper_2309_05315_amd import mam
    monkeypatch.setenv("MAM_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    probs = inputs.batched_problems(n=10, k_range=(8, 20), iters=10)
    scheds = autotune.tune_batch(probs, iters=2, warm=1)
    b = mam.Batch(probs, schedules=scheds)
    assert b.groups() == len(scheds)
    b.init()
    b.iterate(10)
    for i, p in enumerate(probs):
        ref = O.mam([p.cost_block(m) for m in range(p.M)], [p.q_block(m) for m in range(p.M)], p.rho, p.gamma, 10)["p_bar"]
        got = b.barycenter(i).cpu().numpy()
        assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-5
