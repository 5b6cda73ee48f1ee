"""HIP path vs the FP64 oracle at each workload's stated iteration count
(MI355X only).

The references under tests/golden/fullk/ were written by
tests/golden/make_fullk_refs.py, which runs only the oracle (Alg. 1 in the
paper's scheme of one process per group of measures, equal bit for bit to
the one-process oracle) on the seeded generators of
``paper_2309_05315_amd.inputs``; a hash of the regenerated inputs must match
the one stored with each reference.

Gates, with tol = 1e-5 for FP32 plans and 1e-10 for FP64 plans:
* the barycenter p_bar: relative L1 and max norms <= tol;
* the marginals p^(m) of theta^K: max |diff| / max |p^(m)| <= tol;
* W_hat = sum_m <c^(m), pi_hat^(m)> of the last iteration: relative <= tol;
* dist_L(pi_hat) of the last iteration: the device forms it from the row
  sums of pi_hat, p^(m),K + t (p - p^(m),K-1), each within tol max|p^(m)| by
  the marginal gate, so |diff| <= 4 tol max|p^(m)| sqrt(R sum_m 1/S^m);
* the measure residual max |sum_r pi_hat_rs - q_s|: <= 1e-12 max q on both;
* the damping t of the last iteration: relative <= tol.
"""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

from paper_2309_05315_amd import mam

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullk_refs as refs  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
INDEX = json.load(open(refs.INDEX)) if os.path.exists(refs.INDEX) else {}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def load(name):
    meta = INDEX[name]
    arr = np.load(os.path.join(refs.OUT, name + ".npz"))
    return meta, arr["p_bar"], arr["pm"]


def rel(a, b, ord=1):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    if ord == 1:
        return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_every_reference_is_present():
    names = set(refs.workloads())
    missing = sorted(names - set(INDEX))
    assert not missing, f"references not written: {missing}"
    for n in names:
        assert os.path.exists(os.path.join(refs.OUT, n + ".npz")), n


SINGLE = [n for n in refs.workloads() if not n.startswith("batch")]


@pytest.mark.parametrize("name", SINGLE)
def test_full_iteration_count(name):
    build, iters, what = refs.workloads()[name]
    meta, pbar_o, pm_o = load(name)
    p = build()
    assert refs.inputs_hash(p) == meta["inputs_sha256"], "the generator changed since the reference was written"
    assert meta["iters"] == iters
    tol = TOL[p.dtype]
    say(f"case {name}: R={p.R} M={p.M} T={p.T} {iters} iterations ({what})")
    s = mam.solver_for(p, diag=True)
    s.init()
    s.iterate(iters)
    d = s.diagnostics()
    pbar = s.barycenter().cpu().numpy()
    pm = s.marginals().cpu().numpy()
    s.close()
    e1, einf = rel(pbar, pbar_o), rel(pbar, pbar_o, np.inf)
    epm = float(np.abs(pm - pm_o).max() / np.abs(pm_o).max())
    eW = abs(d["W_hat"] - meta["W_hat"])
    dist_bound = 4 * tol * np.abs(pm_o).max() * math.sqrt(p.R * sum(1.0 / s_ for s_ in p.S))
    edist = abs(d["dist_L"] - meta["dist_L"])
    et = abs(d["t"] - meta["t_last"]) / meta["t_last"]
    say(f"  p_bar rel L1 {e1:.3e} max {einf:.3e}; marginals rel max {epm:.3e}; "
        f"W_hat {d['W_hat']:.10e} vs {meta['W_hat']:.10e} (rel {eW / max(abs(meta['W_hat']), 1e-300):.2e}); "
        f"dist_L {d['dist_L']:.6e} vs {meta['dist_L']:.6e} (|diff| {edist:.2e}, bound {dist_bound:.2e}); "
        f"meas_resid {d['meas_resid']:.1e} / {meta['meas_resid']:.1e}; t {d['t']:.6g} rel {et:.1e}")
    assert e1 <= tol and einf <= tol
    assert epm <= tol
    assert eW <= tol * abs(meta["W_hat"])   # a zero objective (all mass on zero-cost entries) must stay 0
    assert edist <= dist_bound
    qmax = float(np.abs(p.q).max())
    assert d["meas_resid"] <= 1e-12 * qmax and meta["meas_resid"] <= 1e-12 * qmax
    assert et <= tol


def test_batch_of_256_full_iteration_count():
    """The 256-problem batch (configs of uneven R, M), 300 iterations in one
    plan with graph replay; the sampled problems against their references."""
    from paper_2309_05315_amd import inputs
    names = [n for n in refs.workloads() if n.startswith("batch")]
    iters = refs.workloads()[names[0]][1]
    probs = inputs.batched_problems(iters=iters)
    b = mam.Batch(probs)
    b.graph(50)
    b.init()
    b.iterate(iters)
    torch.cuda.synchronize()
    for name in names:
        meta, pbar_o, _ = load(name)
        i = int(name.split("_p")[1].split("_")[0])
        p = probs[i]
        assert refs.inputs_hash(p) == meta["inputs_sha256"]
        got = b.barycenter(i).cpu().numpy()
        e1, einf = rel(got, pbar_o), rel(got, pbar_o, np.inf)
        say(f"  problem {i} {p.name} (group {b.group_of(i)}): {iters} iterations, rel L1 {e1:.3e} max {einf:.3e}")
        assert e1 <= TOL["f32"] and einf <= TOL["f32"]
    b.close()
