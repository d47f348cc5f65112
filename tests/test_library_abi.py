"""The C-ABI library loads and exports every entry point include/rfeig.h declares.

Runs on the CPU: no compute call is made, only symbol lookup, the pure host
helpers (option defaults, status strings) and argument checks that fail before
any device work.
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
    assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # r <= 0
    o.w = 1; o.r = 0.0
    assert lib.rf_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(o), None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # bad column index
    o.r = 1.0
    badcol = np.array([0, 5], dtype=np.int32)
    Ab = rfeig.RfCsr(2, 2, rowptr.ctypes.data, badcol.ctypes.data, val.ctypes.data)
    assert lib.rf_plan_create(ctypes.byref(Ab), ctypes.byref(A), ctypes.byref(o), None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    # non-finite value
    nanval = np.array([float("nan"), 0.0, 2.0, 0.0])
    An = rfeig.RfCsr(2, 2, rowptr.ctypes.data, col.ctypes.data, nanval.ctypes.data)
    assert lib.rf_plan_create(ctypes.byref(An), ctypes.byref(A), ctypes.byref(o), None,
                              ctypes.byref(out)) == rfeig.RF_ERR_ARG
    assert out.value is None
