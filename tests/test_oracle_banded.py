"""Pins of the oracle's band LU and band solves.

Independent references: LAPACK's band solver (scipy.linalg.solve_banded, i.e.
gbsv) and dense LU (numpy.linalg.solve); plus the backward-error bound of
partial-pivoting LU and the exact-zero-pivot detection.
"""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import banded

RNG = np.random.default_rng(7)


def _random_band(n, kl, ku, zero_diag=False):
    M = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(max(0, i - kl), min(n, i + ku + 1)):
            M[i, j] = RNG.standard_normal() + 1j * RNG.standard_normal()
    if zero_diag:
        np.fill_diagonal(M, 0.0)
    return M


@pytest.mark.parametrize("n,kl,ku", [(1, 0, 0), (7, 0, 0), (40, 3, 5), (41, 5, 3),
                                     (64, 1, 1), (100, 16, 16), (33, 0, 4), (33, 4, 0),
                                     (130, 20, 7)])
def test_band_solve_matches_lapack_and_dense(n, kl, ku):
    M = _random_band(n, kl, ku)
    f = banded.band_lu(sp.csr_matrix(M), kl, ku)
    assert f.info == 0
    Bm = RNG.standard_normal((n, 3)) + 1j * RNG.standard_normal((n, 3))
    x = f.solve(Bm)
    # LAPACK gbsv via scipy (band storage of the upper/lower parts)
    ab = np.zeros((kl + ku + 1, n), dtype=np.complex128)
    for i in range(n):
        for j in range(max(0, i - kl), min(n, i + ku + 1)):
            ab[ku + i - j, j] = M[i, j]
    x_lapack = sl.solve_banded((kl, ku), ab, Bm)
    x_dense = np.linalg.solve(M, Bm)
    scale = np.linalg.norm(x_dense)
    assert np.linalg.norm(x - x_lapack) <= 1e-11 * scale
    assert np.linalg.norm(x - x_dense) <= 1e-11 * scale
    # backward error of partial pivoting LU
    r = np.linalg.norm(M @ x - Bm) / (np.linalg.norm(M, 1) * np.linalg.norm(x) + np.linalg.norm(Bm))
    assert r <= 50 * np.finfo(float).eps


def test_pivoting_required_zero_diagonal():
    n, kl, ku = 60, 2, 2
    M = _random_band(n, kl, ku, zero_diag=True)
    f = banded.band_lu(sp.csr_matrix(M), kl, ku)
    assert f.info == 0
    assert np.any(f.ipiv != np.arange(n))
    b = RNG.standard_normal(n) + 0j
    x = f.solve(b)
    assert np.linalg.norm(M @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_exact_zero_pivot_reported():
    M = np.diag(np.array([1.0, 2.0, 0.0, 4.0], dtype=np.complex128))
    f = banded.band_lu(sp.csr_matrix(M), 1, 1)
    assert f.info == 3


def test_vector_and_block_agree():
    n, kl, ku = 50, 4, 2
    M = _random_band(n, kl, ku)
    f = banded.band_lu(sp.csr_matrix(M), kl, ku)
    b = RNG.standard_normal((n, 2)) + 1j
    assert np.array_equal(f.solve(b)[:, 1], f.solve(b[:, 1]))


def test_bandwidths():
    M = sp.diags([np.ones(9), np.ones(10), np.ones(7)], [-1, 0, 3], shape=(10, 10))
    assert banded.bandwidths(M) == (1, 3)
