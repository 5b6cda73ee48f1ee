"""Python binding of libmam.so (ctypes): argument marshalling only.

Every step of the iteration runs in the HIP kernels behind the C ABI of
``include/mam.h``; torch supplies device memory and the stream.  There is
no CPU path: if the library is missing, ``lib()`` raises.

Names follow the paper: R (barycenter support size), S (columns S^m of each
plan), rho (DR prox parameter), gamma (unbalanced penalty, inf = balanced),
q (measure weights), theta (the DR iterate), p (barycenter).
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

__all__ = ["lib", "MAMError", "Solver", "Batch", "solver_for", "solve_static", "stream_copy", "cost_sq_euclid",
           "F32", "F64", "COST_PER_COLUMN", "COST_SHARED", "COST_INDEXED", "COST_GRID", "FLAG_DIAG", "FLAG_COLD", "FLAG_RELAXED", "FLAG_SPARSE_STORE",
           "STOP_TESTS", "EXPORTED"]

F32, F64 = 0, 1
COST_PER_COLUMN, COST_SHARED, COST_INDEXED, COST_GRID = 0, 1, 2, 3
FLAG_DIAG, FLAG_COLD, FLAG_RELAXED, FLAG_SPARSE_STORE = 1, 2, 4, 8
# stopping tests of Sec. 5 (MAM_STOP_*)
STOP_TESTS = {"dtheta": 0, "dp": 1, "dist": 2}

STATUS = {0: "MAM_OK", -1: "MAM_EINVAL", -2: "MAM_ENOMEM", -3: "MAM_EHIP",
          -4: "MAM_ENOTBALANCED", -5: "MAM_ENONFINITE", -6: "MAM_EUNSUPPORTED",
          -7: "MAM_ESTATE"}

EXPORTED = ["mam_abi_version", "mam_last_error", "mam_create", "mam_set_schedule",
            "mam_get_schedule", "mam_workspace_bytes", "mam_set_workspace", "mam_bind",
            "mam_init", "mam_iterate", "mam_barycenter", "mam_barycenter_host",
            "mam_marginals", "mam_diagnostics", "mam_timing_enable", "mam_timing_read",
            "mam_destroy", "mam_cost_sq_euclid", "mam_graph", "mam_batch_create",
            "mam_batch_groups", "mam_batch_group_of", "mam_batch_set_schedule",
            "mam_batch_get_schedule", "mam_batch_workspace_bytes", "mam_batch_set_workspace",
            "mam_batch_bind", "mam_batch_init", "mam_batch_iterate", "mam_batch_graph",
            "mam_batch_barycenter", "mam_batch_timing_enable", "mam_batch_timing_read",
            "mam_batch_destroy", "mam_adjoint_workspace_bytes", "mam_record", "mam_backward",
            "mam_bundle_workspace_bytes", "mam_set_bundles", "mam_iterate_bundles",
            "mam_iterate_until", "mam_set_grid", "mam_support_workspace_bytes", "mam_support_update",
            "mam_solve_static", "mam_stream_copy"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmam.so")


class Desc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("cost_mode", ctypes.c_int32),
                ("R", ctypes.c_int64), ("M", ctypes.c_int64),
                ("S", ctypes.POINTER(ctypes.c_int64)), ("ld", ctypes.c_int64),
                ("cost_ld", ctypes.c_int64), ("cost_ncols", ctypes.c_int64),
                ("rho", ctypes.c_double), ("gamma", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


class Diag(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("t", ctypes.c_double),
                ("W_hat", ctypes.c_double), ("dist_L", ctypes.c_double),
                ("meas_resid", ctypes.c_double), ("dtheta_inf", ctypes.c_double),
                ("dp_norm", ctypes.c_double), ("p_mass", ctypes.c_double),
                ("rounds_per_column", ctypes.c_double), ("active_per_column", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("threads_per_column", ctypes.c_int32), ("values_per_thread", ctypes.c_int32),
                ("columns_in_flight", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("vector_width", ctypes.c_int32),
                ("order", ctypes.c_int32), ("streaming", ctypes.c_int32),
                ("rows_per_tile", ctypes.c_int32), ("candidate_slots", ctypes.c_int32),
                ("team_size", ctypes.c_int32)]


class StopResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("checks", ctypes.c_int64),
                ("converged", ctypes.c_int32), ("value", ctypes.c_double)]


class MAMError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_LIB = None
_vp = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load libmam.so from this package directory (raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2309_05315_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "mam_abi_version": (ctypes.c_int32, []),
        "mam_last_error": (ctypes.c_char_p, []),
        "mam_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.POINTER(Desc)]),
        "mam_set_schedule": (ctypes.c_int32, [_vp, ctypes.POINTER(Schedule)]),
        "mam_get_schedule": (ctypes.c_int32, [_vp, ctypes.POINTER(Schedule)]),
        "mam_workspace_bytes": (ctypes.c_size_t, [_vp]),
        "mam_set_workspace": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t]),
        "mam_bind": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _vp]),
        "mam_init": (ctypes.c_int32, [_vp, _vp, _vp]),
        "mam_iterate": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp]),
        "mam_barycenter": (ctypes.c_int32, [_vp, _vp, _vp]),
        "mam_barycenter_host": (ctypes.c_int32, [_vp, _vp, _vp]),
        "mam_marginals": (ctypes.c_int32, [_vp, _vp, _vp]),
        "mam_diagnostics": (ctypes.c_int32, [_vp, ctypes.POINTER(Diag), _vp]),
        "mam_timing_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
        "mam_timing_read": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int64)]),
        "mam_destroy": (None, [_vp]),
        "mam_cost_sq_euclid": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, ctypes.c_int64,
                                                ctypes.c_int32, ctypes.c_int32, _vp,
                                                ctypes.c_int64, ctypes.c_int32, _vp, _vp]),
        "mam_graph": (ctypes.c_int32, [_vp, ctypes.c_int64]),
        "mam_batch_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.POINTER(Desc), ctypes.c_int32]),
        "mam_batch_groups": (ctypes.c_int32, [_vp]),
        "mam_batch_group_of": (ctypes.c_int32, [_vp, ctypes.c_int32]),
        "mam_batch_set_schedule": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(Schedule)]),
        "mam_batch_get_schedule": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(Schedule)]),
        "mam_batch_workspace_bytes": (ctypes.c_size_t, [_vp]),
        "mam_batch_set_workspace": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t]),
        "mam_batch_bind": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp]),
        "mam_batch_init": (ctypes.c_int32, [_vp, _vp]),
        "mam_batch_iterate": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp]),
        "mam_batch_graph": (ctypes.c_int32, [_vp, ctypes.c_int64]),
        "mam_batch_barycenter": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp]),
        "mam_batch_timing_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
        "mam_batch_timing_read": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_int64)]),
        "mam_batch_destroy": (None, [_vp]),
        "mam_adjoint_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int64, ctypes.c_int64]),
        "mam_record": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int64, _vp, ctypes.c_size_t, _vp]),
        "mam_backward": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _vp]),
        "mam_bundle_workspace_bytes": (ctypes.c_size_t, [_vp, _vp, ctypes.c_int32]),
        "mam_set_bundles": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
        "mam_iterate_bundles": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp]),
        "mam_set_grid": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
        "mam_support_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
        "mam_support_update": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp,
                                                ctypes.c_size_t, _vp]),
        "mam_iterate_until": (ctypes.c_int32, [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_int64, ctypes.POINTER(StopResult), _vp]),
        "mam_stream_copy": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp]),
        "mam_solve_static": (ctypes.c_int32, [ctypes.POINTER(Desc), _vp, _vp, _vp, _vp, _vp, ctypes.c_int64,
                                              _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _check(code: int, where: str) -> None:
    if code != 0:
        raise MAMError(code, where, lib().mam_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _round_up(x: int, k: int) -> int:
    return (x + k - 1) // k * k


class Solver:
    """One MAM problem on one GPU: a handle, its workspace and bound buffers.

    theta: (T, ld) tensor, row j = plan column j (column-major R x T plans).
    cost:  (ncols, cost_ld) tensor, row k = cost column k.
    q:     (T,) tensor of the weights of every measure, concatenated.
    """

    def __init__(self, R: int, S: Sequence[int], rho: float = 1.0, gamma: float = math.inf,
                 dtype: torch.dtype = torch.float32, cost_mode: int = COST_SHARED,
                 cost_ncols: Optional[int] = None, ld: Optional[int] = None,
                 cost_ld: Optional[int] = None, diag: bool = False, cold: bool = False,
                 relaxed: bool = False, sparse_store: bool = False,
                 threads_per_column: int = 0, columns_in_flight: int = 0,
                 workgroups: int = 0, xcd_remap: int = 0, order: int = 0, streaming: int = 0,
                 rows_per_tile: int = 0, candidate_slots: int = 0, team_size: int = 0, device="cuda"):
        L = lib()
        self.device = torch.device(device)
        self.R, self.S = int(R), [int(s) for s in S]
        self.M, self.T = len(self.S), int(sum(self.S))
        self.dtype = dtype
        vec = 4 if dtype == torch.float32 else 2
        self.ld = int(ld) if ld else _round_up(self.R, vec)
        self.cost_ld = int(cost_ld) if cost_ld else _round_up(self.R, vec)
        if cost_ncols is None:
            cost_ncols = self.T if cost_mode == COST_PER_COLUMN else max(self.S)
        self.cost_ncols = int(cost_ncols)
        self.cost_mode = cost_mode
        self._S_arr = (ctypes.c_int64 * self.M)(*self.S)
        d = Desc(dtype=F32 if dtype == torch.float32 else F64, cost_mode=cost_mode,
                 R=self.R, M=self.M, S=self._S_arr, ld=self.ld, cost_ld=self.cost_ld,
                 cost_ncols=self.cost_ncols, rho=float(rho), gamma=float(gamma),
                 flags=(FLAG_DIAG if diag else 0) | (FLAG_COLD if cold else 0) | (FLAG_RELAXED if relaxed else 0)
                 | (FLAG_SPARSE_STORE if sparse_store else 0))
        h = _vp()
        _check(L.mam_create(ctypes.byref(h), ctypes.byref(d)), "mam_create")
        self._h = h
        if (threads_per_column or columns_in_flight or workgroups or xcd_remap or order or streaming
                or rows_per_tile or candidate_slots or team_size):
            sc = Schedule(threads_per_column=threads_per_column, columns_in_flight=columns_in_flight,
                          workgroups=workgroups, xcd_remap=xcd_remap, order=order, streaming=streaming,
                          rows_per_tile=rows_per_tile, candidate_slots=candidate_slots, team_size=team_size)
            _check(L.mam_set_schedule(h, ctypes.byref(sc)), "mam_set_schedule")
        nbytes = int(L.mam_workspace_bytes(h))
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _check(L.mam_set_workspace(h, _ptr(self.workspace), nbytes), "mam_set_workspace")
        self.theta = self.cost = self.q = self.index = None

    # -- buffers -----------------------------------------------------------
    def bind(self, theta: torch.Tensor, cost: torch.Tensor, q: torch.Tensor,
             index: Optional[torch.Tensor] = None) -> None:
        grid = self.cost_mode == COST_GRID
        for name, t in (("theta", theta), ("cost", cost), ("q", q)):
            want = torch.float64 if (grid and name == "cost") else self.dtype
            if t.dtype != want or t.device.type != "cuda" or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {want} CUDA tensor")
        if theta.shape != (self.T, self.ld):
            raise ValueError(f"theta must have shape {(self.T, self.ld)}")
        if grid:
            if cost.dim() != 2 or cost.shape[0] != self.cost_ncols or cost.shape[1] not in (1, 2):
                raise ValueError(f"grid cost: the measures' points, shape ({self.cost_ncols}, dim)")
        elif cost.shape != (self.cost_ncols, self.cost_ld):
            raise ValueError(f"cost must have shape {(self.cost_ncols, self.cost_ld)}")
        if q.shape != (self.T,):
            raise ValueError(f"q must have shape {(self.T,)}")
        if index is not None and (index.dtype != torch.int32 or index.shape != (self.T,)):
            raise ValueError("index must be an int32 tensor of length T")
        self.theta, self.cost, self.q, self.index = theta, cost, q, index
        _check(lib().mam_bind(self._h, _ptr(theta), _ptr(cost), _ptr(index), _ptr(q)), "mam_bind")

    def schedule(self) -> dict:
        sc = Schedule()
        _check(lib().mam_get_schedule(self._h, ctypes.byref(sc)), "mam_get_schedule")
        return {k: getattr(sc, k) for k, _ in Schedule._fields_}

    def set_grid(self, n: Sequence[int], origin: Sequence[float], spacing: Sequence[float]) -> None:
        """Barycenter support of a COST_GRID problem: a regular grid with n[k]
        points per axis at origin[k] + i * spacing[k] (last axis fastest)."""
        d = len(n)
        _check(lib().mam_set_grid(self._h, d, (ctypes.c_int64 * d)(*[int(x) for x in n]),
                                  (ctypes.c_double * d)(*[float(x) for x in origin]),
                                  (ctypes.c_double * d)(*[float(x) for x in spacing])), "mam_set_grid")

    # -- iteration ---------------------------------------------------------
    def init(self, theta0: Optional[torch.Tensor] = None) -> None:
        _check(lib().mam_init(self._h, _ptr(theta0), _stream(self.device)), "mam_init")

    def iterate(self, iters: int) -> None:
        _check(lib().mam_iterate(self._h, int(iters), _stream(self.device)), "mam_iterate")

    def iterate_until(self, max_iters: int, test: str = "dtheta", tol: float = 1e-8,
                      check_every: int = 1) -> dict:
        """Iterate until a stopping test of Sec. 5 holds ("dtheta", "dp" or
        "dist", evaluated on the device every check_every iterations), at
        most max_iters iterations.  Blocks until the run ends; returns
        {"iterations", "checks", "converged", "value"}."""
        if test not in STOP_TESTS:
            raise ValueError(f"unknown stopping test {test!r}; one of {sorted(STOP_TESTS)}")
        r = StopResult()
        _check(lib().mam_iterate_until(self._h, int(max_iters), STOP_TESTS[test], float(tol), int(check_every),
                                       ctypes.byref(r), _stream(self.device)), "mam_iterate_until")
        return {"iterations": r.iterations, "checks": r.checks, "converged": bool(r.converged),
                "value": r.value}

    def barycenter(self) -> torch.Tensor:
        out = torch.empty(self.R, dtype=torch.float64, device=self.device)
        _check(lib().mam_barycenter(self._h, _ptr(out), _stream(self.device)), "mam_barycenter")
        return out

    def marginals(self) -> torch.Tensor:
        out = torch.empty(self.M, self.R, dtype=torch.float64, device=self.device)
        _check(lib().mam_marginals(self._h, _ptr(out), _stream(self.device)), "mam_marginals")
        return out

    def diagnostics(self) -> dict:
        d = Diag()
        _check(lib().mam_diagnostics(self._h, ctypes.byref(d), _stream(self.device)),
               "mam_diagnostics")
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def graph(self, iters_per_launch: int) -> None:
        """Replay iterations from a captured HIP graph (0 = off)."""
        _check(lib().mam_graph(self._h, int(iters_per_launch)), "mam_graph")

    def timing(self, enable: bool) -> None:
        _check(lib().mam_timing_enable(self._h, int(enable)), "mam_timing_enable")

    def timing_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().mam_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)), "mam_timing_read")
        return ms.value, n.value

    # -- randomized variant --------------------------------------------------
    def set_bundles(self, bundle_of: Sequence[int]) -> None:
        """Partition the measures into bundles (bundle_of[m] = bundle of measure m)."""
        arr = (ctypes.c_int32 * self.M)(*[int(b) for b in bundle_of])
        nb = max(int(b) for b in bundle_of) + 1
        n = int(lib().mam_bundle_workspace_bytes(self._h, arr, nb))
        if n == 0:
            raise MAMError(-1, "mam_bundle_workspace_bytes", "invalid partition")
        self.bundle_workspace = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().mam_set_bundles(self._h, arr, nb, _ptr(self.bundle_workspace), n, _stream(self.device)),
               "mam_set_bundles")

    def iterate_bundles(self, seq: Sequence[int]) -> None:
        """One randomized iteration per entry of seq (the bundle it updates)."""
        s = np.ascontiguousarray(np.asarray(seq, dtype=np.int32))
        _check(lib().mam_iterate_bundles(self._h, int(s.size), s.ctypes.data_as(_vp), _stream(self.device)),
               "mam_iterate_bundles")

    # -- support step (Prop. 4) ---------------------------------------------
    def support_update(self, alpha: Sequence[float], zeta: torch.Tensor, xi: torch.Tensor):
        """Run one more iteration, then move the support points to the
        alpha-weighted means of the measures' points under that iteration's
        plans (rows without mass keep theirs).  zeta: (T, dim) float64 on
        the device, the point of each plan column; xi: (R, dim) float64 on
        the device, updated in place.  Returns (xi, mass)."""
        if zeta.dtype != torch.float64 or xi.dtype != torch.float64:
            raise ValueError("points must be float64")
        if zeta.dim() != 2 or xi.dim() != 2 or zeta.shape != (self.T, xi.shape[1]) or xi.shape[0] != self.R:
            raise ValueError(f"zeta must be ({self.T}, dim) and xi ({self.R}, dim)")
        if not (zeta.is_contiguous() and xi.is_contiguous()):
            raise ValueError("zeta and xi must be contiguous")
        dim = int(xi.shape[1])
        al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
        if al.shape != (self.M,):
            raise ValueError(f"alpha must hold {self.M} weights")
        n = int(lib().mam_support_workspace_bytes(self._h, dim))
        if n == 0:
            raise MAMError(-1, "mam_support_workspace_bytes", f"invalid dimension {dim}")
        if getattr(self, "support_workspace", None) is None or self.support_workspace.numel() < n:
            self.support_workspace = torch.empty(n, dtype=torch.uint8, device=self.device)
        mass = torch.empty(self.R, dtype=torch.float64, device=self.device)
        _check(lib().mam_support_update(self._h, al.ctypes.data_as(_vp), _ptr(zeta), dim, _ptr(xi), _ptr(mass),
                                        _ptr(self.support_workspace), self.support_workspace.numel(),
                                        _stream(self.device)), "mam_support_update")
        return xi, mass

    # -- reverse mode --------------------------------------------------------
    def record(self, iters: int, ckpt_every: int = 0) -> None:
        """Run 'iters' iterations (after a default init) keeping what backward() needs."""
        n = int(lib().mam_adjoint_workspace_bytes(self._h, int(iters), int(ckpt_every)))
        if n == 0:
            raise MAMError(-1, "mam_adjoint_workspace_bytes", "no reverse mode for these arguments")
        self.adj_workspace = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().mam_record(self._h, int(iters), int(ckpt_every), _ptr(self.adj_workspace), n,
                                _stream(self.device)), "mam_record")

    def backward(self, grad_p: torch.Tensor):
        """dL/dq (T,) and dL/dcost (cost_ncols, cost_ld) for dL/dp_bar = grad_p."""
        gp = grad_p.detach().to(device=self.device, dtype=torch.float64).contiguous()
        if gp.shape != (self.R,):
            raise ValueError(f"grad_p must have shape {(self.R,)}")
        gq = torch.empty(self.T, dtype=self.dtype, device=self.device)
        gc = torch.zeros(self.cost_ncols, self.cost_ld, dtype=self.dtype, device=self.device)
        _check(lib().mam_backward(self._h, _ptr(gp), _ptr(gq), _ptr(gc), _stream(self.device)),
               "mam_backward")
        return gq, gc

    def plans(self) -> list:
        """theta^(m) as R x S^m float64 numpy arrays (copies, for checking)."""
        th = self.theta[:, :self.R].double().cpu().numpy()
        off = np.concatenate([[0], np.cumsum(self.S)])
        return [th[off[m]:off[m + 1]].T.copy() for m in range(self.M)]

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().mam_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solver_for(problem, device="cuda", diag: bool = False, cold: bool = False, relaxed: bool = False,
               sparse_store: bool = False, grid: bool = False, **sched) -> Solver:
    """Allocate device buffers for an ``inputs.Problem`` and bind them
    (sparse_store: on long columns, keep the plans as -b plus the active
    entries between the iterations of a call, MAM_FLAG_SPARSE_STORE)
    (relaxed: measure constraints sum_r pi_rs <= q_s, with the problem's
    cost taken as the shifted c - eta; grid: a problem whose support is a
    regular grid (meta["grid"]) forms its cost in the kernels from the
    points instead of storing it)."""
    dt = torch.float32 if problem.dtype == "f32" else torch.float64
    ncols = problem.cost_ncols
    if grid:
        mode = COST_GRID
    elif problem.col_index is None:
        mode = COST_SHARED
    elif np.array_equal(problem.col_index, np.arange(problem.T)):
        mode = COST_PER_COLUMN
    else:
        mode = COST_INDEXED
    s = Solver(problem.R, problem.S, rho=problem.rho, gamma=problem.gamma, dtype=dt,
               cost_mode=mode, cost_ncols=ncols, diag=diag, cold=cold, relaxed=relaxed,
               sparse_store=sparse_store, device=device, **sched)
    if grid:
        n, origin, spacing = problem.meta["grid"]
        s.set_grid(n, origin, spacing)
        cost = torch.from_numpy(np.ascontiguousarray(problem.zeta, dtype=np.float64)).to(device)
    elif problem.cost is None:
        # a cost given by its points is built on the device (rounded once to dt)
        cost = cost_sq_euclid(torch.from_numpy(problem.xi).to(device), torch.from_numpy(problem.zeta).to(device),
                              dtype=dt, ld=s.cost_ld)
    else:
        cost = torch.zeros(ncols, s.cost_ld, dtype=dt)
        cost[:, :problem.R] = torch.from_numpy(problem.cost).to(dt)
        cost = cost.to(device)
    theta = torch.zeros(problem.T, s.ld, dtype=dt, device=device)
    idx = None
    if mode == COST_INDEXED:
        idx = torch.from_numpy(problem.col_index.astype(np.int32)).to(device)
    s.bind(theta, cost, torch.from_numpy(problem.q).to(dt).to(device), idx)
    return s


def solve_static(R: int, S: Sequence[int], theta: torch.Tensor, cost: torch.Tensor, q: torch.Tensor,
                 iters: int, rho: float = 1.0, gamma: float = math.inf, cost_mode: int = COST_SHARED,
                 index: Optional[torch.Tensor] = None, theta0: Optional[torch.Tensor] = None,
                 cost_ncols: Optional[int] = None, flags: int = 0,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One whole solve (init, ``iters`` iterations, barycenter) on the
    library's static workspace (mam_solve_static): no workspace is
    allocated.  Buffers as for ``Solver.bind`` (theta is written and holds
    theta^iters on return); returns p_bar (R doubles on theta's device)."""
    S = [int(s) for s in S]
    dt = theta.dtype
    if cost_ncols is None:
        cost_ncols = sum(S) if cost_mode == COST_PER_COLUMN else max(S)
    S_arr = (ctypes.c_int64 * len(S))(*S)
    d = Desc(dtype=F32 if dt == torch.float32 else F64, cost_mode=cost_mode, R=int(R), M=len(S), S=S_arr,
             ld=int(theta.shape[1]), cost_ld=int(cost.shape[1]), cost_ncols=int(cost_ncols),
             rho=float(rho), gamma=float(gamma), flags=int(flags))
    if out is None:
        out = torch.empty(int(R), dtype=torch.float64, device=theta.device)
    _check(lib().mam_solve_static(ctypes.byref(d), _ptr(theta), _ptr(cost), _ptr(index), _ptr(q), _ptr(theta0),
                                  int(iters), _ptr(out), _stream(theta.device)), "mam_solve_static")
    return out


def stream_copy(dst: torch.Tensor, src: torch.Tensor, workgroups: int) -> None:
    """Device copy with the library's bandwidth probe (mam_stream_copy)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(lib().mam_stream_copy(_ptr(dst), _ptr(src), nbytes, int(workgroups), _stream(src.device)),
           "mam_stream_copy")


def _dtype_of(problem):
    return torch.float32 if problem.dtype == "f32" else torch.float64


def _cost_mode_of(problem):
    if problem.col_index is None:
        return COST_SHARED
    if np.array_equal(problem.col_index, np.arange(problem.T)):
        return COST_PER_COLUMN
    return COST_INDEXED


def _device_buffers(problem, ld, cost_ld, dt, device):
    """theta (zeros), cost and q (and the index for an indexed cost) on the device."""
    mode = _cost_mode_of(problem)
    ncols = problem.cost.shape[0]
    cost = torch.zeros(ncols, cost_ld, dtype=dt)
    cost[:, :problem.R] = torch.from_numpy(problem.cost).to(dt)
    theta = torch.zeros(problem.T, ld, dtype=dt, device=device)
    idx = None
    if mode == COST_INDEXED:
        idx = torch.from_numpy(problem.col_index.astype(np.int32)).to(device)
    q = torch.from_numpy(problem.q).to(dt).to(device)
    return theta, cost.to(device), q, idx


class Batch:
    """Many independent problems advanced together (one launch per shape
    group per iteration, optionally replayed from a HIP graph)."""

    def __init__(self, problems, device="cuda", schedules=None):
        L = lib()
        self.device = torch.device(device)
        self.problems = list(problems)
        dts = {p.dtype for p in self.problems}
        if len(dts) != 1:
            raise ValueError("all problems of a batch share one dtype")
        self.dtype = _dtype_of(self.problems[0])
        vec = 4 if self.dtype == torch.float32 else 2
        descs = (Desc * len(self.problems))()
        self._S = []
        self.lds = []
        for i, p in enumerate(self.problems):
            S = (ctypes.c_int64 * p.M)(*p.S)
            self._S.append(S)
            ld = _round_up(p.R, vec)
            self.lds.append(ld)
            descs[i] = Desc(dtype=F32 if self.dtype == torch.float32 else F64, cost_mode=_cost_mode_of(p),
                            R=p.R, M=p.M, S=S, ld=ld, cost_ld=ld, cost_ncols=p.cost.shape[0],
                            rho=float(p.rho), gamma=float(p.gamma), flags=0)
        h = _vp()
        _check(L.mam_batch_create(ctypes.byref(h), descs, len(self.problems)), "mam_batch_create")
        self._h = h
        for g, sc in (schedules or {}).items():
            s = Schedule(**sc)
            _check(L.mam_batch_set_schedule(h, int(g), ctypes.byref(s)), "mam_batch_set_schedule")
        nbytes = int(L.mam_batch_workspace_bytes(h))
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _check(L.mam_batch_set_workspace(h, _ptr(self.workspace), nbytes), "mam_batch_set_workspace")
        self.buffers = []
        for i, p in enumerate(self.problems):
            theta, cost, q, idx = _device_buffers(p, self.lds[i], self.lds[i], self.dtype, self.device)
            self.buffers.append((theta, cost, q, idx))
            _check(L.mam_batch_bind(h, i, _ptr(theta), _ptr(cost), _ptr(idx), _ptr(q)), "mam_batch_bind")

    def group_of(self, i: int) -> int:
        """Shape group of problem i."""
        return int(lib().mam_batch_group_of(self._h, int(i)))

    def groups(self) -> int:
        return int(lib().mam_batch_groups(self._h))

    def schedule(self, group: int) -> dict:
        sc = Schedule()
        _check(lib().mam_batch_get_schedule(self._h, int(group), ctypes.byref(sc)), "mam_batch_get_schedule")
        return {k: getattr(sc, k) for k, _ in Schedule._fields_}

    def init(self) -> None:
        _check(lib().mam_batch_init(self._h, _stream(self.device)), "mam_batch_init")

    def iterate(self, iters: int) -> None:
        _check(lib().mam_batch_iterate(self._h, int(iters), _stream(self.device)), "mam_batch_iterate")

    def graph(self, iters_per_launch: int) -> None:
        _check(lib().mam_batch_graph(self._h, int(iters_per_launch)), "mam_batch_graph")

    def barycenter(self, i: int) -> torch.Tensor:
        out = torch.empty(self.problems[i].R, dtype=torch.float64, device=self.device)
        _check(lib().mam_batch_barycenter(self._h, int(i), _ptr(out), _stream(self.device)),
               "mam_batch_barycenter")
        return out

    def plans(self, i: int) -> list:
        p = self.problems[i]
        th = self.buffers[i][0][:, :p.R].double().cpu().numpy()
        off = np.concatenate([[0], np.cumsum(p.S)])
        return [th[off[m]:off[m + 1]].T.copy() for m in range(p.M)]

    def timing(self, enable: bool) -> None:
        _check(lib().mam_batch_timing_enable(self._h, int(enable)), "mam_batch_timing_enable")

    def timing_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().mam_batch_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)),
               "mam_batch_timing_read")
        return ms.value, n.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().mam_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cost_sq_euclid(xi: torch.Tensor, zeta: torch.Tensor, normalize_max: bool = False,
                   dtype: torch.dtype = torch.float64, ld: Optional[int] = None) -> torch.Tensor:
    """||xi_r - zeta_s||^2 on the GPU as an (S, ld) tensor (row s = cost column s)."""
    if xi.dtype != torch.float64 or zeta.dtype != torch.float64:
        raise ValueError("points must be float64")
    R, dim = xi.shape
    S = zeta.shape[0]
    ld = int(ld) if ld else R
    out = torch.zeros(S, ld, dtype=dtype, device=xi.device)
    scratch = torch.empty(1, dtype=torch.float64, device=xi.device)
    _check(lib().mam_cost_sq_euclid(_ptr(xi.contiguous()), R, _ptr(zeta.contiguous()), S, dim,
                                    int(normalize_max), _ptr(out), ld,
                                    F32 if dtype == torch.float32 else F64, _ptr(scratch),
                                    _stream(xi.device)), "mam_cost_sq_euclid")
    return out
