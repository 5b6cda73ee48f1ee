"""The C-ABI library loads, exports every declared symbol, and validates its
arguments before touching the GPU (CPU only: no compute call is made)."""
import ctypes
import math
import os
import re

import pytest

from paper_2309_05315_amd import mam

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "mam.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mam_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = mam.lib()
    decl = declared_functions()
    assert len(decl) >= 18
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(mam.EXPORTED) == decl
    assert L.mam_abi_version() == 1


def desc(**kw):
    S = kw.pop("S", [5, 7])
    arr = (ctypes.c_int64 * len(S))(*S)
    d = mam.Desc(dtype=kw.pop("dtype", mam.F64), cost_mode=kw.pop("cost_mode", mam.COST_PER_COLUMN),
                 R=kw.pop("R", 16), M=len(S), S=arr, ld=kw.pop("ld", 0), cost_ld=kw.pop("cost_ld", 0),
                 cost_ncols=kw.pop("cost_ncols", sum(S)), rho=kw.pop("rho", 1.0),
                 gamma=kw.pop("gamma", math.inf), flags=kw.pop("flags", 0))
    assert not kw
    return d, arr


def create(**kw):
    d, arr = desc(**kw)
    h = ctypes.c_void_p()
    rc = mam.lib().mam_create(ctypes.byref(h), ctypes.byref(d))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(R=0), -1), (dict(S=[3, 0]), -1), (dict(rho=0.0), -1), (dict(rho=-2.0), -1),
    (dict(rho=math.inf), -1), (dict(gamma=-1.0), -1), (dict(gamma=math.nan), -1),
    (dict(dtype=7), -1), (dict(cost_mode=9), -1), (dict(ld=8), -1), (dict(cost_ld=3), -1),
    (dict(cost_mode=mam.COST_SHARED, cost_ncols=5), -1),
    (dict(cost_ncols=3), -1), (dict(R=(1 << 28) + 1), -6),
])
def test_create_rejects(kw, code):
    rc, h = create(**kw)
    assert rc == code
    assert not h.value
    assert mam.lib().mam_last_error()


def test_create_accepts_and_sizes_workspace():
    L = mam.lib()
    rc, h = create(R=300, S=[40, 1, 17])
    assert rc == 0 and h.value
    n = L.mam_workspace_bytes(h)
    assert n > 0 and n % 256 == 0
    sc = mam.Schedule()
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0
    assert sc.threads_per_column == 64 and sc.values_per_thread == 8   # double, R = 300
    # workspace checks are pure pointer/size checks
    assert L.mam_set_workspace(h, ctypes.c_void_p(0x100000 + 8), n) == -1
    assert L.mam_set_workspace(h, ctypes.c_void_p(0x100000), n - 1) == -2
    assert L.mam_set_workspace(h, None, n) == -2
    # out-of-order calls
    assert L.mam_iterate(h, 1, None) == -7
    assert L.mam_init(h, None, None) == -7
    assert L.mam_bind(h, None, None, None, None) == -1
    L.mam_destroy(h)
    L.mam_destroy(None)


def test_schedule_override_validation():
    L = mam.lib()
    rc, h = create(R=4096, S=[100])
    assert rc == 0
    bad = mam.Schedule(threads_per_column=100)
    assert L.mam_set_schedule(h, ctypes.byref(bad)) == -1
    small = mam.Schedule(threads_per_column=64)     # 4096 rows at 64 threads = 64 values per lane
    assert L.mam_set_schedule(h, ctypes.byref(small)) == -6
    tiny = mam.Schedule(threads_per_column=128)     # 32 values per thread
    assert L.mam_set_schedule(h, ctypes.byref(tiny)) == -6
    kc3 = mam.Schedule(columns_in_flight=3)
    assert L.mam_set_schedule(h, ctypes.byref(kc3)) == -1
    ok = mam.Schedule(threads_per_column=1024, columns_in_flight=4, workgroups=37, xcd_remap=-1)
    assert L.mam_set_schedule(h, ctypes.byref(ok)) == 0
    sc = mam.Schedule()
    L.mam_get_schedule(h, ctypes.byref(sc))
    assert (sc.threads_per_column, sc.values_per_thread, sc.columns_in_flight, sc.workgroups,
            sc.xcd_remap) == (1024, 4, 4, 37, 0)
    assert sc.streaming == -1                       # 100 columns of 4096 doubles stay cached
    bad_stream = mam.Schedule(streaming=2)
    assert L.mam_set_schedule(h, ctypes.byref(bad_stream)) == -1
    on = mam.Schedule(streaming=1)
    assert L.mam_set_schedule(h, ctypes.byref(on)) == 0
    L.mam_get_schedule(h, ctypes.byref(sc))
    assert sc.streaming == 1
    L.mam_destroy(h)
    # plans of 4096 x 10,000 doubles (328 MB) are streamed by default
    rc, h = create(R=4096, S=[5000, 5000])
    L.mam_get_schedule(h, ctypes.byref(sc))
    assert sc.streaming == 1
    L.mam_destroy(h)


def test_indexed_mode_requires_index():
    L = mam.lib()
    rc, h = create(cost_mode=mam.COST_INDEXED, cost_ncols=4)
    assert rc == 0
    fake = ctypes.c_void_p(0x200000)
    assert L.mam_bind(h, fake, fake, None, fake) == -1
    rc2, h2 = create()
    assert L.mam_bind(h2, fake, fake, fake, fake) == -1       # index given in per-column mode
    assert L.mam_bind(h2, ctypes.c_void_p(0x200001), fake, None, fake) == -1   # misaligned
    assert L.mam_bind(h2, fake, fake, None, fake) == 0
    L.mam_destroy(h)
    L.mam_destroy(h2)


def test_cost_helper_validation():
    L = mam.lib()
    fake = ctypes.c_void_p(0x300000)
    assert L.mam_cost_sq_euclid(None, 4, fake, 4, 2, 0, fake, 4, 1, None, None) == -1
    assert L.mam_cost_sq_euclid(fake, 4, fake, 4, 2, 0, fake, 3, 1, None, None) == -1
    assert L.mam_cost_sq_euclid(fake, 4, fake, 4, 2, 1, fake, 4, 1, None, None) == -1
    assert L.mam_cost_sq_euclid(fake, 4, fake, 4, 2, 0, fake, 4, 5, None, None) == -1


def test_reverse_mode_validation():
    L = mam.lib()
    assert L.mam_adjoint_workspace_bytes(None, 10, 0) == 0
    rc, h = create(R=300, S=[40, 1, 17])
    assert rc == 0
    assert L.mam_adjoint_workspace_bytes(h, -1, 0) == 0
    full = L.mam_adjoint_workspace_bytes(h, 10, 0)
    assert full > 0 and full % 256 == 0
    # ckpt_every beyond the run keeps every mask, like 0
    assert L.mam_adjoint_workspace_bytes(h, 10, 50) == full
    # windows of 3 iterations: 4 mask slots instead of 11, plus 3 checkpoints of theta
    assert L.mam_adjoint_workspace_bytes(h, 10, 3) != full
    fake = ctypes.c_void_p(0x100000)
    assert L.mam_record(None, 10, 0, fake, full, None) == -1
    assert L.mam_record(h, 10, 0, fake, full, None) == -7       # no init yet
    assert L.mam_backward(None, fake, fake, fake, None) == -1
    assert L.mam_backward(h, fake, fake, fake, None) == -7      # no record yet
    L.mam_destroy(h)


def test_bundle_validation():
    L = mam.lib()
    rc, h = create(R=50, S=[10, 20, 30])
    assert rc == 0
    B3 = ctypes.c_int32 * 3
    assert L.mam_bundle_workspace_bytes(None, B3(0, 1, 2), 3) == 0
    assert L.mam_bundle_workspace_bytes(h, B3(0, 3, 1), 3) == 0        # index out of range
    assert L.mam_bundle_workspace_bytes(h, B3(0, 0, 2), 3) == 0        # bundle 1 is empty
    assert L.mam_bundle_workspace_bytes(h, B3(0, 1, 0), 2) > 0
    fake = ctypes.c_void_p(0x100000)
    assert L.mam_set_bundles(None, B3(0, 1, 0), 2, fake, 1 << 20, None) == -1
    assert L.mam_set_bundles(h, B3(0, 1, 0), 2, fake, 1 << 20, None) == -7   # no init yet
    assert L.mam_iterate_bundles(h, 1, None, None) == -7
    L.mam_destroy(h)


def test_stopping_test_validation():
    L = mam.lib()
    rc, h = create(R=40, S=[10, 20])
    assert rc == 0
    r = mam.StopResult()
    assert L.mam_iterate_until(None, 5, 0, 1e-3, 1, ctypes.byref(r), None) == -1
    assert L.mam_iterate_until(h, 5, 0, 1e-3, 1, None, None) == -1           # no result struct
    assert L.mam_iterate_until(h, 5, 0, 1e-3, 1, ctypes.byref(r), None) == -7  # no init yet
    assert r.iterations == 0 and r.checks == 0 and r.converged == 0 and math.isnan(r.value)
    L.mam_destroy(h)


def test_long_column_path_selection():
    L = mam.lib()
    sc = mam.Schedule()
    # single problems with R > 8192 take the long-column path
    rc, h = create(R=10000, S=[30, 20])
    assert rc == 0
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0
    assert sc.rows_per_tile == 2048 and sc.candidate_slots == 64   # double
    assert L.mam_workspace_bytes(h) > 0
    assert L.mam_adjoint_workspace_bytes(h, 10, 0) == 0                    # no reverse mode
    B2 = ctypes.c_int32 * 2
    assert L.mam_bundle_workspace_bytes(h, B2(0, 1), 2) == 0               # no randomized variant
    bad = mam.Schedule(rows_per_tile=1000)
    assert L.mam_set_schedule(h, ctypes.byref(bad)) == -1
    ok = mam.Schedule(rows_per_tile=1024, candidate_slots=8)
    assert L.mam_set_schedule(h, ctypes.byref(ok)) == 0
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0
    assert sc.rows_per_tile == 1024 and sc.values_per_thread == 4 and sc.candidate_slots == 8
    L.mam_destroy(h)
    # forced on a short problem, and back
    rc, h = create(R=300, S=[40, 17])
    assert rc == 0
    assert L.mam_set_schedule(h, ctypes.byref(mam.Schedule(rows_per_tile=1024))) == 0
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0 and sc.rows_per_tile == 1024
    assert L.mam_set_schedule(h, ctypes.byref(mam.Schedule())) == 0
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0 and sc.rows_per_tile == 0
    L.mam_destroy(h)
    # batches keep R <= 8192
    d, arr = desc(R=9000, S=[10])
    ds = (mam.Desc * 1)(d)
    b = ctypes.c_void_p()
    assert L.mam_batch_create(ctypes.byref(b), ds, 1) == -6


def test_grid_cost_validation():
    L = mam.lib()
    rc, h = create(R=12, S=[5, 5], cost_mode=mam.COST_GRID, cost_ncols=5)
    assert rc == 0
    sc = mam.Schedule()
    assert L.mam_get_schedule(h, ctypes.byref(sc)) == 0 and sc.rows_per_tile > 0   # long-column path
    N2, D2 = ctypes.c_int64 * 2, ctypes.c_double * 2
    assert L.mam_set_grid(h, 2, N2(3, 5), D2(0, 0), D2(1, 1)) == -1     # 15 points, R = 12
    assert L.mam_set_grid(h, 3, N2(3, 4), D2(0, 0), D2(1, 1)) == -1     # dim 3
    assert L.mam_set_grid(h, 2, N2(3, 4), D2(0, float("nan")), D2(1, 1)) == -1
    assert L.mam_set_grid(h, 2, N2(3, 4), D2(0, 0), D2(0.5, 0.25)) == 0
    L.mam_destroy(h)
    rc, h = create(R=12, S=[5], cost_mode=mam.COST_SHARED, cost_ncols=5)
    assert L.mam_set_grid(h, 1, (ctypes.c_int64 * 1)(12), (ctypes.c_double * 1)(0), (ctypes.c_double * 1)(1)) == -1
    L.mam_destroy(h)
    d, arr = desc(R=12, S=[5], cost_mode=mam.COST_GRID, cost_ncols=5)
    b = ctypes.c_void_p()
    assert L.mam_batch_create(ctypes.byref(b), (mam.Desc * 1)(d), 1) == -6


def test_support_step_validation():
    L = mam.lib()
    fake = ctypes.c_void_p(0x400000)
    alpha = (ctypes.c_double * 2)(0.5, 0.5)
    assert L.mam_support_workspace_bytes(None, 2) == 0
    assert L.mam_support_update(None, alpha, fake, 2, fake, None, fake, 1 << 20, None) == -1
    rc, h = create(R=300, S=[40, 17])
    assert rc == 0
    assert L.mam_support_workspace_bytes(h, 0) == 0 and L.mam_support_workspace_bytes(h, 4) == 0
    n1, n2, n3 = (L.mam_support_workspace_bytes(h, d) for d in (1, 2, 3))
    # chunk tables plus (dim + 1) partial sums per row and chunk
    # 2 chunks here: each dimension adds 2 * R doubles (up to the 256-byte alignment)
    assert 0 < n1 < n2 < n3 and n2 - n1 > 2 * 300 * 8 - 256 and n3 - n2 > 2 * 300 * 8 - 256
    assert L.mam_support_update(h, alpha, fake, 2, fake, None, fake, n2, None) == -7   # no init yet
    L.mam_destroy(h)


def test_sparse_store_workspace():
    """The sparse store adds, on long columns only, the patch slots (a count,
    and per slot a row and a value) per (column, sub-tile) and two halves of
    the common values per (measure, row)."""
    L = mam.lib()
    sizes = {}
    for R in (300, 10000):
        for fl in (0, mam.FLAG_SPARSE_STORE):
            rc, h = create(R=R, S=[30, 20], flags=fl)
            assert rc == 0
            sizes[R, fl] = L.mam_workspace_bytes(h)
            L.mam_destroy(h)
    assert sizes[300, 0] == sizes[300, mam.FLAG_SPARSE_STORE]
    # R = 10000 in FP64: 2048-row tiles, 5 tiles of 4 sub-tiles, 64 slots
    nh = 50 * 5 * 4
    extra = nh * 4 + nh * 64 * (4 + 8) + 2 * 2 * 10000 * 8 + 4
    grown = sizes[10000, mam.FLAG_SPARSE_STORE] - sizes[10000, 0]
    assert extra <= grown <= extra + 5 * 256


def test_solve_static_rejects_before_touching_the_gpu():
    """mam_solve_static checks its arguments and the workspace size before
    any HIP call, so these run without a GPU (the pointers below are never
    dereferenced: every call returns before the buffers are bound)."""
    L = mam.lib()
    fake = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p(0x200000)
    d, arr = desc(R=64, S=[64, 64], cost_mode=mam.COST_SHARED, cost_ncols=64)
    assert L.mam_solve_static(None, fake, fake, None, fake, None, 5, out, None) == -1
    assert L.mam_solve_static(ctypes.byref(d), None, fake, None, fake, None, 5, out, None) == -1
    assert L.mam_solve_static(ctypes.byref(d), fake, fake, None, fake, None, 5, None, None) == -1
    assert L.mam_solve_static(ctypes.byref(d), fake, fake, None, fake, None, -1, out, None) == -1
    g, garr = desc(R=64, S=[64], cost_mode=mam.COST_GRID, cost_ncols=64)
    assert L.mam_solve_static(ctypes.byref(g), fake, fake, None, fake, None, 5, out, None) == -6
    bad, barr = desc(R=0, S=[3])
    assert L.mam_solve_static(ctypes.byref(bad), fake, fake, None, fake, None, 5, out, None) == -1
    # 8192 rows, 1024 measures: the marginals alone (three M x R double arrays) exceed the 128 MiB array
    big, bigarr = desc(R=8192, S=[2] * 1024, dtype=mam.F32, cost_mode=mam.COST_SHARED, cost_ncols=2)
    hb = ctypes.c_void_p()
    assert L.mam_create(ctypes.byref(hb), ctypes.byref(big)) == 0
    assert L.mam_workspace_bytes(hb) > (128 << 20)
    L.mam_destroy(hb)
    assert L.mam_solve_static(ctypes.byref(big), fake, fake, None, fake, None, 5, out, None) == -2
    assert b"static workspace" in L.mam_last_error()
