"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments before touching the GPU (host-only paths; no device needed)."""

import ctypes as C
import os
import re

import pytest

from paper_2409_03030_amd import wdirac as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wdirac.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wd_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = W.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps exactly the declared calls
    assert sorted(W.SYMBOLS) == names


def test_lattice_argument_checks():
    lib = W.lib()
    h = C.c_void_p()
    ok = (C.c_int32 * 4)(4, 4, 4, 4)
    bc = (C.c_int32 * 4)(1, 1, 1, -1)
    assert lib.wd_lattice_create(C.byref(h), ok, bc) == W.WD_OK
    odd = (C.c_int32 * 4)(4, 3, 4, 4)
    h2 = C.c_void_p()
    assert lib.wd_lattice_create(C.byref(h2), odd, bc) == W.WD_EINVAL
    assert b"even" in lib.wd_last_error()
    badbc = (C.c_int32 * 4)(1, 1, 1, 0)
    assert lib.wd_lattice_create(C.byref(h2), ok, badbc) == W.WD_EINVAL
    # gauge store sizes: V sites x 4 links x bytes per link
    V = 256
    assert lib.wd_gauge_bytes(h, W.F64, 18) == V * 4 * 18 * 8
    assert lib.wd_gauge_bytes(h, W.F64, 12) == V * 4 * 12 * 8
    assert lib.wd_gauge_bytes(h, W.F32, 18) == V * 4 * 18 * 4
    assert lib.wd_gauge_bytes(h, W.F32, 12) == V * 4 * 12 * 4
    assert lib.wd_gauge_bytes(h, W.F16, 12) == V * 4 * 12 * 2
    assert lib.wd_gauge_bytes(h, W.F16, 18) == V * 4 * 18 * 2
    assert lib.wd_gauge_bytes(h, W.F64, 13) == 0
    # apply before set_gauge: no gauge store
    dummy = C.c_void_p(0x1000)
    st = lib.wd_apply_D(h, dummy, dummy, 1, 0.1, 0, W.EO, W.F64, dummy, 1 << 30, None)
    assert st == W.WD_ENOGAUGE
    # solve with bad parameters
    p = W.default_params()
    p.tol = -1.0
    stats = (W.SolveStats * 1)()
    k = (C.c_double * 1)(0.1)
    assert lib.wd_solve_DdagD(h, dummy, dummy, 1, k, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_EINVAL
    p = W.default_params()
    assert lib.wd_solve_DdagD(h, dummy, dummy, 1, k, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_ENOGAUGE
    assert lib.wd_lattice_destroy(h) == W.WD_OK


def test_solve_D_and_pion_argument_checks():
    lib = W.lib()
    h = C.c_void_p()
    assert lib.wd_lattice_create(C.byref(h), (C.c_int32 * 4)(4, 4, 4, 8), (C.c_int32 * 4)(1, 1, 1, -1)) == W.WD_OK
    dummy = C.c_void_p(256)
    p = W.default_params()
    stats = (W.SolveStats * 1)()
    k = (C.c_double * 1)(0.1)
    assert lib.wd_solve_D(h, None, dummy, 1, k, 0, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_EINVAL
    assert lib.wd_solve_D(h, dummy, dummy, 1, k, 2, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_EINVAL
    assert lib.wd_solve_D(h, dummy, dummy, 0, k, 0, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_EINVAL
    assert lib.wd_solve_D(h, dummy, dummy, 1, k, 0, C.byref(p), dummy, 1 << 30, stats, None) == W.WD_ENOGAUGE
    n1 = lib.wd_solve_D_workspace_bytes(h, C.byref(p), 1)
    n4 = lib.wd_solve_D_workspace_bytes(h, C.byref(p), 4)
    # the D^dag D solve's workspace plus the boundary-layout source and FP64 fields
    assert n1 > lib.wd_solver_workspace_bytes(h, C.byref(p), 1) + 4 * 4 * 4 * 8 * 12 * 16
    assert n4 > 3 * n1
    corr = (C.c_double * 8)()
    nw = lib.wd_pion_workspace_bytes(h)
    assert nw >= 8 * 8
    assert lib.wd_pion_correlator(h, corr, dummy, 12, 8, dummy, nw, None) == W.WD_EINVAL   # t0 = Lt
    assert lib.wd_pion_correlator(h, corr, dummy, 12, -1, dummy, nw, None) == W.WD_EINVAL
    assert lib.wd_pion_correlator(h, corr, dummy, 0, 0, dummy, nw, None) == W.WD_EINVAL
    assert lib.wd_pion_correlator(h, corr, dummy, 12, 0, dummy, nw - 1, None) == W.WD_EBUFSIZE
    assert lib.wd_pion_correlator(h, None, dummy, 12, 0, dummy, nw, None) == W.WD_EINVAL
    assert lib.wd_lattice_destroy(h) == W.WD_OK


def test_force_argument_checks():
    lib = W.lib()
    h = C.c_void_p()
    assert lib.wd_lattice_create(C.byref(h), (C.c_int32 * 4)(4, 4, 4, 4), (C.c_int32 * 4)(1, 1, 1, -1)) == W.WD_OK
    dummy = C.c_void_p(256)
    p = W.default_params()
    stats = (W.SolveStats * 2)()
    act = C.c_double()
    big = 1 << 30
    assert lib.wd_fermion_force(h, None, None, dummy, 0.1, C.byref(p), dummy, big, stats, None) == W.WD_EINVAL
    assert lib.wd_fermion_force(h, dummy, C.byref(act), None, 0.1, C.byref(p), dummy, big, stats, None) == W.WD_EINVAL
    assert lib.wd_fermion_force(h, dummy, C.byref(act), dummy, float("nan"), C.byref(p), dummy, big, stats,
                                None) == W.WD_EINVAL
    assert lib.wd_fermion_force(h, dummy, C.byref(act), dummy, 0.1, C.byref(p), dummy, big, stats, None) == W.WD_ENOGAUGE
    n = lib.wd_fermion_force_workspace_bytes(h, C.byref(p))
    assert n > lib.wd_solve_D_workspace_bytes(h, C.byref(p), 1) + 2 * 4 ** 4 * 192
    assert lib.wd_ta_add(h, None, 0.1, dummy, None) == W.WD_EINVAL
    assert lib.wd_ta_add(h, dummy, float("inf"), dummy, None) == W.WD_EINVAL
    assert lib.wd_lattice_destroy(h) == W.WD_OK


def test_staggered_argument_checks():
    lib = W.lib()
    h = C.c_void_p()
    assert lib.wd_lattice_create(C.byref(h), (C.c_int32 * 4)(4, 4, 4, 4), (C.c_int32 * 4)(1, 1, 1, -1)) == W.WD_OK
    dummy = C.c_void_p(256)
    big = 1 << 30
    assert lib.wd_stag_apply(h, dummy, dummy, 1, 0.1, 0, W.F16, dummy, big, None) == W.WD_EINVAL
    assert lib.wd_stag_apply(h, dummy, dummy, 1, 0.1, 2, W.F64, dummy, big, None) == W.WD_EINVAL
    assert lib.wd_stag_apply(h, dummy, dummy, 1, 0.1, 0, W.F64, dummy, big, None) == W.WD_ENOGAUGE
    assert lib.wd_stag_apply_workspace_bytes(h, W.F64, 2) == 2 * lib.wd_stag_apply_workspace_bytes(h, W.F64, 1)
    p = W.default_params()
    stats = (W.SolveStats * 1)()
    m = (C.c_double * 1)(0.1)
    zero = (C.c_double * 1)(0.0)
    assert lib.wd_stag_solve(h, dummy, dummy, 1, m, 0, C.byref(p), dummy, big, stats, None) == W.WD_ENOGAUGE
    pf = W.default_params(precond="full")
    assert lib.wd_stag_solve(h, dummy, dummy, 1, m, 0, C.byref(pf), dummy, big, stats, None) == W.WD_EINVAL
    p16 = W.default_params(inner="f16")
    assert lib.wd_stag_solve(h, dummy, dummy, 1, m, 0, C.byref(p16), dummy, big, stats, None) == W.WD_EINVAL
    assert lib.wd_stag_solve(h, dummy, dummy, 1, zero, 0, C.byref(p), dummy, big, stats, None) in (W.WD_EINVAL,
                                                                                                  W.WD_ENOGAUGE)
    assert lib.wd_stag_set_shape(h, W.F64, 1, 128, 0, 1) == W.WD_ENOGAUGE
    assert lib.wd_stag_set_shape(h, W.F16, 1, 128, 0, 1) == W.WD_EINVAL
    nw = lib.wd_pion_workspace_bytes(h)
    corr = (C.c_double * 4)()
    assert lib.wd_stag_pion_correlator(h, corr, dummy, 3, 4, dummy, nw, None) == W.WD_EINVAL   # t0 = Lt
    assert lib.wd_stag_pion_correlator(h, corr, dummy, 0, 0, dummy, nw, None) == W.WD_EINVAL
    assert lib.wd_stag_pion_correlator(h, corr, dummy, 3, 0, dummy, nw - 1, None) == W.WD_EBUFSIZE
    assert lib.wd_stag_pion_correlator(h, corr, None, 3, 0, dummy, nw, None) == W.WD_EINVAL
    n1 = lib.wd_stag_solve_workspace_bytes(h, C.byref(p), 1)
    # a colour vector is a quarter of a Wilson spinor
    assert 0 < n1 < lib.wd_solver_workspace_bytes(h, C.byref(p), 1) + 4 ** 4 * 200
    assert lib.wd_lattice_destroy(h) == W.WD_OK


def test_default_params():
    p = W.default_params()
    assert p.tol == 1e-10 and p.inner == W.F64 and p.precond == W.EO and p.use_graph == 1


def test_workspace_sizes_scale_with_nrhs():
    lib = W.lib()
    lat = W.Lattice((8, 8, 8, 8))
    p = W.default_params()
    a1 = lib.wd_solver_workspace_bytes(lat.handle, C.byref(p), 1)
    a12 = lib.wd_solver_workspace_bytes(lat.handle, C.byref(p), 12)
    assert a12 > 10 * a1 // 2
    w1 = lib.wd_apply_workspace_bytes(lat.handle, W.F64, 1)
    # 4 full-lattice vectors of 24 doubles per site
    assert w1 >= 4 * 8 ** 4 * 24 * 8


def test_tuning_table_roundtrip():
    lib = W.lib()
    assert lib.wd_tune_import(b"16 16 16 32 0 18 1 64 1 2\n24 24 24 48 1 12 12 16 0 1\n") == W.WD_OK
    n = lib.wd_tune_export(None, 0)
    buf = C.create_string_buffer(n)
    lib.wd_tune_export(buf, n)
    txt = buf.value.decode()
    assert "16 16 16 32 0 18 1 64 1 2" in txt
    assert "24 24 24 48 1 12 12 16 0 1" in txt
    assert lib.wd_tune_import(b"1 2 3\n") == W.WD_EINVAL
    assert lib.wd_tune_import(b"16 16 16 32 0 18 1 3 1 1\n") == W.WD_EINVAL   # not a power of two
    assert lib.wd_tune_import(b"16 16 16 32 0 18 1 128 1 4\n") == W.WD_EINVAL  # 512 threads
    assert lib.wd_tune_import(b"16 16 16 32 0 18 1 64 1 3\n") == W.WD_EINVAL   # split 3
    assert lib.wd_tune_import(b"16 16 16 32 1 12 1 64 1 8\n") == W.WD_OK       # 8-way split, FP32
    assert lib.wd_tune_import(b"16 16 16 32 0 12 1 64 1 8\n") == W.WD_EINVAL   # not at FP64


def test_status_strings():
    lib = W.lib()
    for s in range(-8, 1):
        assert lib.wd_status_string(s)
    assert b"gfx950" in lib.wd_version()
