"""Schedule autotuner for the column kernel.

A schedule (threads per column, columns in flight, workgroups, column order,
XCD remap) changes only speed, never results beyond summation order.  The
tuner times candidate schedules on the device with the library's own
column-kernel timing (HIP events on the launch stream) and keeps the
fastest.  Results are cached in a JSON file under a key of the problem's
shape: dtype, cost mode, R, M, the S^m list and the number of cost columns.

    sched = autotune.tune(problem)                  # kwargs for mam.solver_for
    scheds = autotune.tune_batch(problems)          # {group: schedule} for mam.Batch

Schedules of 16 or 32 threads per column (sub-wave groups) compute no
diagnostics; tune without them (threads_per_column >= 64 candidates) for a
solver that will run with diag=True or the reverse mode.

Cache file: $MAM_AUTOTUNE_CACHE, else ~/.cache/paper_2309_05315_amd/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional

import torch

from . import mam

__all__ = ["tune", "tune_batch", "problem_key", "cache_path", "candidates"]


def cache_path() -> str:
    env = os.environ.get("MAM_AUTOTUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2309_05315_amd", "autotune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    data = _load()
    data[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home: tuning still works, it is just not remembered


def problem_key(p) -> str:
    mode = mam._cost_mode_of(p)
    s_hash = hashlib.sha1(",".join(str(int(s)) for s in p.S).encode()).hexdigest()[:12]
    return f"{p.dtype}|mode{mode}|R{p.R}|M{p.M}|S{s_hash}|ncols{p.cost.shape[0]}"


def _default_threads(p) -> int:
    target = 16 if p.dtype == "f32" else 8
    nt = 64
    while nt < 1024 and nt * target < p.R:
        nt *= 2
    return nt


def candidates(p, wide: bool = True) -> List[dict]:
    """Schedules to try: the default threads per column and its neighbours,
    one or two columns in flight, and (wide) the column order, XCD remap and
    two workgroup counts.  Short columns (one wave per column by default)
    also try sub-wave groups of 16 and 32 lanes.  The workgroup counts are
    the default (one resident wave of workgroups), 512 and 1024 (two resident
    waves for the one-wave shapes, which balances columns of uneven cost);
    batch groups keep one resident wave (tune_batch).
    Invalid ones are rejected by the library and skipped."""
    nt0 = _default_threads(p)
    nts = [nt for nt in (nt0 // 2, nt0, nt0 * 2) if 64 <= nt <= 1024]
    if nt0 == 64:
        nts = [16, 32] + nts
    orders = [1, 2] if (wide and mam._cost_mode_of(p) != mam.COST_PER_COLUMN) else [0]
    xcds = [1, -1] if wide else [0]
    wgs = [0, 512, 1024] if wide else [0]
    out = []
    for nt in nts:
        for kc in ((1,) if nt < 64 else (1, 2)):
            for order in orders:
                for xcd in xcds:
                    for wg in wgs:
                        out.append({"threads_per_column": nt, "columns_in_flight": kc, "order": order,
                                    "xcd_remap": xcd, "workgroups": wg})
    return out


def _time_solver(p, sched: dict, iters: int, warm: int) -> Optional[float]:
    try:
        s = mam.solver_for(p, **sched)
    except mam.MAMError:
        return None
    try:
        s.init()
        s.iterate(warm)
        s.timing(True)
        s.iterate(iters)
        ms, n = s.timing_read()
        return ms / max(n, 1)
    finally:
        s.close()
        del s
        torch.cuda.empty_cache()


def tune(p, iters: int = 6, warm: int = 2, use_cache: bool = True, wide: bool = True,
         cands: Optional[Iterable[dict]] = None) -> dict:
    """Fastest schedule for one problem, as keyword arguments of mam.solver_for."""
    key = "single|" + problem_key(p)
    if use_cache and cands is None:
        hit = _load().get(key)
        if hit:
            return dict(hit["schedule"])
    best, best_ms, trials = None, float("inf"), []
    for sc in (cands if cands is not None else candidates(p, wide)):
        ms = _time_solver(p, sc, iters, warm)
        trials.append((sc, ms))
        if ms is not None and ms < best_ms:
            best, best_ms = sc, ms
    if best is None:
        raise RuntimeError("no candidate schedule ran")
    if cands is None:
        _store(key, {"schedule": best, "column_ms": best_ms, "trials": len(trials)})
    return dict(best)


def _time_batch(problems, group_sched: dict, iters: int, warm: int) -> Optional[float]:
    try:
        b = mam.Batch(problems, schedules={0: group_sched})
    except mam.MAMError:
        return None
    try:
        b.init()
        b.iterate(warm)
        b.timing(True)
        b.iterate(iters)
        ms, n = b.timing_read()
        return ms / max(n, 1)
    finally:
        b.close()
        del b
        torch.cuda.empty_cache()


def tune_batch(problems, iters: int = 6, warm: int = 2, use_cache: bool = True) -> Dict[int, dict]:
    """Fastest schedule of every shape group of mam.Batch(problems): each group
    is tuned on a batch of its own problems (groups run as separate launches)."""
    probe = mam.Batch(problems)
    groups: Dict[int, List[int]] = {}
    for i in range(len(problems)):
        groups.setdefault(probe.group_of(i), []).append(i)
    probe.close()
    del probe
    torch.cuda.empty_cache()
    out = {}
    cache = _load() if use_cache else {}
    for g, idx in sorted(groups.items()):
        sub = [problems[i] for i in idx]
        key = "batch|" + hashlib.sha1("|".join(problem_key(p) for p in sub).encode()).hexdigest()[:20]
        if key in cache:
            out[g] = dict(cache[key]["schedule"])
            continue
        nt0 = max(_default_threads(p) for p in sub)
        best, best_ms = None, float("inf")
        for nt in ((16, 32) if nt0 == 64 else ()) + (nt0 // 2, nt0, nt0 * 2):
            if not 16 <= nt <= 1024 or (32 < nt < 64):
                continue
            # one resident wave of workgroups per group: a group tuned alone
            # to two waves (1024) hogs the device inside the batch's graph,
            # where the groups run side by side (0.94 against 0.84 ms per
            # iteration on the 256-problem batch)
            for kc in ((1,) if nt < 64 else (1, 2)):
                for xcd in (1, -1):
                    sc = {"threads_per_column": nt, "columns_in_flight": kc, "xcd_remap": xcd}
                    ms = _time_batch(sub, sc, iters, warm)
                    if ms is not None and ms < best_ms:
                        best, best_ms = sc, ms
        if best is None:
            raise RuntimeError(f"no candidate schedule ran for group {g}")
        out[g] = best
        _store(key, {"schedule": best, "column_ms": best_ms})
    return out
