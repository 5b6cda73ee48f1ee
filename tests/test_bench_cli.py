"""The benchmark's command-line contract on the host: one GPU only, known
workload names, a loud exit without a GPU, and the CPU-baseline record."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args, timeout=120):
    env = dict(os.environ)
    env.pop("WORLD_SIZE", None)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_unknown_workload_is_refused():
    r = run("--extras", "free_support,no_such_workload")
    assert r.returncode == 2 and "--extras" in r.stderr


def test_no_gpu_exits_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the benchmark would run")
    r = run("--no-cpu", "--no-extras", "--no-fp64", "--steps", "1", "--warmup", "0")
    assert r.returncode == 1 and "needs a GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_record():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2309_05315_amd import inputs
    p = inputs.tiny_problem(3, R=40, S=[12, 9, 15], dtype="f32")
    rec = bench.cpu_baseline(p, 2)
    assert set(rec) == {"value", "unit", "cores", "kind", "sample"}
    assert rec["kind"] == "oracle" and rec["cores"] == 1 and rec["value"] > 0
    assert rec["unit"] == "plan-entry updates/s"
    assert "first 2 of 3 measures" in rec["sample"] and f"{40 * 21 * 2:.3e}" in rec["sample"]
    assert "logical cores" in rec["sample"]
