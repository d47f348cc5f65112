"""The C-ABI library loads and exports every entry point include/rfeig.h declares.

Runs on the CPU: no device compute call is made, only symbol lookup, the pure
host helpers (option defaults, status strings, the host QZ of the projected
pencil) and argument checks that fail before any device work.
"""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_18043_amd", "librfeig.so")
HEADER = os.path.join(ROOT, "include", "rfeig.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(rf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import subprocess, sys
        subprocess.check_call([sys.executable, "-m", "paper_2310_18043_amd.build"], cwd=ROOT)
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["rf_plan_create", "rf_factor_shifts", "rf_filter_apply", "rf_solve_region",
              "rf_apply_inner", "rf_plan_destroy", "rf_status_str", "rf_last_error",
              "rf_default_opts"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_status_strings(lib):
    from paper_2310_18043_amd import rfeig  # noqa: F401  (struct layout)
    o = rfeig.RfOpts()
    lib.rf_default_opts(ctypes.byref(o))
    assert (o.p, o.q, o.w) == (4, 8, 32)
    assert o.tau == 1e-10 and o.tau_g == 1e-2 and o.gmres_tol == 1e-12
    assert o.max_subspace_it == 10 and math.isnan(o.sigma_re)
    lib.rf_status_str.restype = ctypes.c_char_p
    for s in range(7):
        assert len(lib.rf_status_str(s)) > 0


def test_plan_create_rejects_bad_arguments_before_device_work(lib):
    from paper_2310_18043_amd import rfeig
    import numpy as np
    o = rfeig.RfOpts()
    lib.rf_default_opts(ctypes.byref(o))
    rowptr = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    val = np.array([1.0, 0.0, 2.0, 0.0])
    A = rfeig.RfCsr(2, 2, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    out = ctypes.c_void_p()
    lib.rf_plan_create.restype = ctypes.c_int
    # w > n
    o.w = 3
    assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None, None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # r <= 0
    o.w = 1; o.r = 0.0
    assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None, None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # bad column index
    o.r = 1.0
    badcol = np.array([0, 5], dtype=np.int32)
    Ab = rfeig.RfCsr(2, 2, rowptr.ctypes.data, badcol.ctypes.data, val.ctypes.data)
    assert lib.rf_plan_create(ctypes.byref(Ab), ctypes.byref(A), ctypes.byref(o), None, None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # non-finite value
    nanval = np.array([float("nan"), 0.0, 2.0, 0.0])
    An = rfeig.RfCsr(2, 2, rowptr.ctypes.data, col.ctypes.data, nanval.ctypes.data)
    assert lib.rf_plan_create(ctypes.byref(An), ctypes.byref(A), ctypes.byref(o), None, None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # tile sizes other than 16, 32, 64, 128, 256
    for bad in (8, 48, 96, 512):
        o.tile = bad
        assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None, None,
                                  ctypes.byref(out)) == rfeig.RF_ERR_ARG
    o.tile = 0
    # precision other than 0 (complex128) and 1 (complex64 band solves)
    for bad in (-1, 2):
        o.precision = bad
        assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None, None,
                                  ctypes.byref(out)) == rfeig.RF_ERR_ARG
    o.precision = 0
    # an allocator must give both callbacks
    half = rfeig.RfAllocator(rfeig.ALLOC_FN(lambda n, ctx: None), rfeig.FREE_FN(), None)
    assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o),
                              ctypes.byref(half), None, ctypes.byref(out)) == rfeig.RF_ERR_ARG
    assert out.value is None


def test_batch_create_rejects_bad_arguments_before_device_work(lib):
    from paper_2310_18043_amd import rfeig
    import numpy as np
    rowptr = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([0, 1], dtype=np.int32)
    val = np.array([1.0, 0.0, 2.0, 0.0])
    A = rfeig.RfCsr(2, 2, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    opts = (rfeig.RfOpts * 2)()
    for d in range(2):
        lib.rf_default_opts(ctypes.byref(opts[d]))
        opts[d].w = 1
    out = ctypes.c_void_p()
    f = lib.rf_batch_create
    f.restype = ctypes.c_int
    # no disks
    assert f(ctypes.byref(A), ctypes.byref(A), opts, 0, None, None, ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # disks that ask for different tiles cannot share one factor storage
    opts[1].tile = 32
    assert f(ctypes.byref(A), ctypes.byref(A), opts, 2, None, None, ctypes.byref(out)) == rfeig.RF_ERR_ARG
    opts[1].tile = 0
    opts[0].p = 0
    assert f(ctypes.byref(A), ctypes.byref(A), opts, 2, None, None, ctypes.byref(out)) == rfeig.RF_ERR_ARG
    assert out.value is None
    lib.rf_batch_size.restype = ctypes.c_int32
    assert lib.rf_batch_size(None) == -1
    lib.rf_batch_plan.restype = ctypes.c_void_p
    assert lib.rf_batch_plan(None, 0) is None


def test_solve_regions_rejects_bad_arguments_before_device_work(lib):
    from paper_2310_18043_amd import rfeig
    f = lib.rf_solve_regions
    f.restype = ctypes.c_int
    res = (rfeig.RfResult * 2)()
    status = (ctypes.c_int * 2)(123, 123)
    assert f(-1, None, 0, None, None, res, status) == rfeig.RF_ERR_ARG
    assert f(2, None, 0, None, None, res, status) == rfeig.RF_ERR_ARG
    # a plan handed in twice would be driven by two threads at once: refused before
    # any handle is touched (these handles are never dereferenced)
    plans = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    assert f(2, plans, 0, None, None, res, status) == rfeig.RF_ERR_ARG
    assert list(status) == [rfeig.RF_ERR_ARG] * 2
    plans = (ctypes.c_void_p * 2)(0x1000, None)
    assert f(2, plans, 1, None, None, res, status) == rfeig.RF_ERR_ARG
    assert f(0, None, 0, None, None, None, None) == rfeig.RF_OK


def _dense_eig(lib, A, B):
    import numpy as np
    f = lib.rf_dense_eig
    f.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 5
    f.restype = ctypes.c_int
    n = A.shape[0]
    A = np.asfortranarray(A, dtype=np.complex128)
    B = np.asfortranarray(B, dtype=np.complex128)
    al = np.zeros(n, np.complex128)
    be = np.zeros(n, np.complex128)
    vr = np.zeros((n, n), np.complex128, order="F")
    st = f(n, A.ctypes.data, B.ctypes.data, al.ctypes.data, be.ctypes.data, vr.ctypes.data)
    return st, al, be, vr


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (128, 4)])
def test_host_qz_matches_lapack_and_residuals(lib, n, seed):
    # the host QZ of HSRR: eigenvalues against LAPACK's generalized eigensolver and
    # ||A v - lambda B v|| small for every returned (unit) vector
    import numpy as np
    import scipy.linalg as sl
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    st, al, be, vr = _dense_eig(lib, A, B)
    assert st == 0
    lam = al / be
    ref = sl.eigvals(A, B)
    d = np.abs(lam[:, None] - ref[None, :])
    from scipy.optimize import linear_sum_assignment
    r, c = linear_sum_assignment(d)
    scale = np.linalg.norm(A, 2) * np.linalg.norm(np.linalg.inv(B), 2)
    assert d[r, c].max() <= 1e-11 * scale, d[r, c].max()
    assert np.allclose(np.linalg.norm(vr, axis=0), 1.0)
    res = np.linalg.norm(A @ vr - (B @ vr) * lam[None, :], axis=0)
    assert res.max() <= 1e-11 * np.linalg.norm(A, 2) * max(1.0, np.abs(lam).max()), res.max()


def test_host_qz_diagonal_and_triangular_pencils(lib):
    # already-triangular input: the eigenvalues are the diagonal ratios exactly
    import numpy as np
    rng = np.random.default_rng(9)
    n = 12
    A = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    B = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
    st, al, be, vr = _dense_eig(lib, A, B)
    assert st == 0
    ref = np.diag(A) / np.diag(B)
    lam = al / be
    assert np.max(np.min(np.abs(lam[:, None] - ref[None, :]), axis=1)) <= 1e-13 * np.abs(ref).max()
