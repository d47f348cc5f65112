"""The host QZ on the swapped pencil that HSRR uses (Sec. 2.1, the eigenpairs of the
projected pencil (A^, B^) = (W^*AV, W^*BV) with W = orth(AV - sigma BV)): since
R = A^ - sigma B^ = W^*(AV - sigma BV) is upper triangular, the QZ runs on (B^, R) with
its QR step skipped, and lambda = sigma + b / a for the pair (a, b) of (B^, R).

The host QZ source is plain C++; it is compiled here with g++ into a small library with
one C entry point, so this runs without a GPU.  Pinned against LAPACK's generalized
eigensolver (scipy) on (A^, B^) directly, and by the residuals ||A^ v - lambda B^ v||."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_18043_amd", "csrc")

SHIM = r'''
#include "rf_qz.h"
extern "C" int qz_ex(int n, const double *A, const double *B, int b_upper, double *al,
                     double *be, double *vr) {
    return host_qz_eig_ex(n, A, B, b_upper != 0, al, be, vr);
}
'''


@pytest.fixture(scope="module")
def qz(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("qz")
    shim = d / "shim.cpp"
    shim.write_text(SHIM)
    lib = d / "libqz_test.so"
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-fcx-limited-range",
                    f"-I{CSRC}", str(shim), os.path.join(CSRC, "rf_qz.cpp"), "-o", str(lib),
                    "-lpthread"], check=True)
    h = ctypes.CDLL(str(lib))
    h.qz_ex.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    h.qz_ex.restype = ctypes.c_int
    return h


def _run(qz, A, B, upper):
    n = A.shape[0]
    A = np.asfortranarray(A, dtype=np.complex128)
    B = np.asfortranarray(B, dtype=np.complex128)
    al = np.zeros(n, np.complex128)
    be = np.zeros(n, np.complex128)
    vr = np.zeros((n, n), np.complex128, order="F")
    st = qz.qz_ex(n, A.ctypes.data, B.ctypes.data, int(upper), al.ctypes.data,
                  be.ctypes.data, vr.ctypes.data)
    return st, al, be, vr


def _pencil(n, sigma, rng, near=None):
    """(A^, B^) with A^ - sigma B^ upper triangular; near: put one eigenvalue at
    sigma + near (a tiny diagonal entry of R)."""
    Bh = np.eye(n) * 3 + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    R = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) + 2 * np.eye(n)
    if near is not None:
        # R e_0 = near B^ e_0 in the first coordinate: lambda = sigma + near exactly
        R[0, 0] = near * Bh[0, 0]
        Bh[1:, 0] = 0.0
    return R + sigma * Bh, Bh, R


def _match(lam, ref):
    from scipy.optimize import linear_sum_assignment
    d = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(d)
    return d[r, c] / np.maximum(np.abs(ref[c]), 1e-300)


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (64, 2), (128, 3)])
def test_swapped_pencil_matches_lapack(qz, n, seed):
    import scipy.linalg as sl
    rng = np.random.default_rng(seed)
    sigma = 2.0 + 0.5j
    Ah, Bh, R = _pencil(n, sigma, rng)
    st, a, b, vr = _run(qz, Bh, R, True)
    assert st == 0
    lam = (sigma * a + b) / a
    ref = sl.eigvals(Ah, Bh)
    rel = _match(lam, ref)
    assert rel.max() <= 1e-11, rel.max()
    # the same eigenvalues as the QZ on (A^, B^) itself
    st2, a2, b2, _ = _run(qz, Ah, Bh, False)
    assert st2 == 0
    assert _match(lam, a2 / b2).max() <= 1e-11
    # unit eigenvectors of the original pencil
    assert np.allclose(np.linalg.norm(vr, axis=0), 1.0)
    res = np.linalg.norm(Ah @ vr - (Bh @ vr) * lam[None, :], axis=0)
    assert res.max() <= 1e-12 * np.linalg.norm(Ah, 2) * max(1.0, np.abs(lam).max()), res.max()


def test_swapped_pencil_eigenvalue_next_to_the_shift(qz):
    # lambda within 1e-9 of sigma: R has a tiny diagonal entry, mu = 1 / (lambda - sigma)
    # is large; lambda must still come out to full relative accuracy
    rng = np.random.default_rng(7)
    sigma = -1.0 + 3.0j
    Ah, Bh, R = _pencil(40, sigma, rng, near=1e-9)
    st, a, b, vr = _run(qz, Bh, R, True)
    assert st == 0
    lam = (sigma * a + b) / a
    k = int(np.argmin(np.abs(lam - sigma)))
    assert abs(lam[k] - (sigma + 1e-9)) <= 1e-13 * abs(sigma), abs(lam[k] - (sigma + 1e-9))
    res = np.linalg.norm(Ah @ vr - (Bh @ vr) * lam[None, :], axis=0)
    assert res.max() <= 1e-12 * np.linalg.norm(Ah, 2) * np.abs(lam).max()


def test_upper_flag_ignores_the_strict_lower_part(qz):
    # with b_upper set, B's strict lower part is never read (taken as zero)
    rng = np.random.default_rng(3)
    n = 16
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    T = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) + 3 * np.eye(n)
    junk = T + np.tril(rng.standard_normal((n, n)), -1) * 1e3
    st1, a1, b1, _ = _run(qz, A, T, True)
    st2, a2, b2, _ = _run(qz, A, junk, True)
    assert st1 == 0 and st2 == 0
    assert np.array_equal(a1 / b1, a2 / b2)
