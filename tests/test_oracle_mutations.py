"""Planted mistakes in the oracle must be caught by its pins.

Each test patches one plausible slip into the oracle (on the CPU only), reruns
the relevant pin's check, and asserts that the check now fails.  This shows
the pins are sensitive to dropped terms, wrong signs or indices and
transposed operands.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import banded, coeffs, filters, hsrr
from paper_2310_18043_amd import workloads as W

RNG = np.random.default_rng(3)


def _compact(z, c, r, k):
    return 1.0 / (1.0 + ((z - c) / r) ** k)


def _compact_error():
    z = 0.3 + 0.2j + 0.05 * RNG.uniform(0, 2.5, 200) * np.exp(2j * np.pi * RNG.uniform(size=200))
    return np.max(np.abs(coeffs.rational_filter(z, 0.3 + 0.2j, 0.05, 8) - _compact(z, 0.3 + 0.2j, 0.05, 8)))


def _composite_error():
    z = 0.05 * RNG.uniform(0, 2.5, 200) * np.exp(2j * np.pi * RNG.uniform(size=200))
    return np.max(np.abs(coeffs.composite_filter(z, 0.0, 0.05, 4, 8) - _compact(z, 0.0, 0.05, 32)))


def _diag_filter_error():
    n, c, r = 40, 0.5, 0.4
    lam = c + r * RNG.uniform(0.1, 2.0, n) * np.exp(2j * np.pi * RNG.uniform(size=n))
    b = RNG.uniform(0.5, 1.5, n)
    A, B = W.diagonal_pencil(lam, b)
    Y = W.start_block(n, 3, 0)
    got = filters.simple_filter(A, B, c, r, 8, Y)
    want = _compact(lam, c, r, 8)[:, None] * Y
    return np.linalg.norm(got - want) / np.linalg.norm(want)


def _band_error():
    n, kl, ku = 40, 3, 2
    M = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for j in range(max(0, i - kl), min(n, i + ku + 1)):
            M[i, j] = RNG.standard_normal() + 1j * RNG.standard_normal()
    np.fill_diagonal(M, 0.1 * np.diag(M))        # forces pivoting
    f = banded.band_lu(sp.csr_matrix(M), kl, ku)
    b = RNG.standard_normal((n, 2)) + 0j
    return np.linalg.norm(M @ f.solve(b) - b) / np.linalg.norm(b)


def _hsrr_error():
    n = 60
    lam = RNG.standard_normal(n) + 1j * RNG.standard_normal(n)
    A, B = W.diagonal_pencil(lam, RNG.uniform(0.5, 1.5, n))
    idx = np.array([2, 9, 33])
    U = np.zeros((n, 3), dtype=complex)
    U[idx, np.arange(3)] = 1.0
    U = U @ (RNG.standard_normal((3, 3)) + 1j * RNG.standard_normal((3, 3)))
    _, got, X = hsrr.hsrr(A, B, U, 0.1j)
    eig_err = np.abs(got[:, None] - lam[idx][None, :]).min(axis=1).max()
    return max(eig_err, hsrr.rel_errors(A, B, got, X, 0.0, 1.0).max())


def test_baselines_are_clean():
    assert _compact_error() < 1e-12
    assert _composite_error() < 1e-11
    assert _diag_filter_error() < 1e-12
    assert _band_error() < 1e-12
    assert _hsrr_error() < 1e-12


def test_wrong_pole_angle_is_caught(monkeypatch):
    def bad(c, r, k):
        i = np.arange(1, k + 1)
        e = np.exp(1j * 2 * i * np.pi / k)          # 2i instead of 2i-1
        return c + r * e, r * e / k
    monkeypatch.setattr(coeffs, "trapezoid_nodes", bad)
    assert _compact_error() > 1e-3


def test_literal_outer_weight_sign_is_caught(monkeypatch):
    good = coeffs.outer_shifts
    monkeypatch.setattr(coeffs, "outer_shifts",
                        lambda q: (lambda s, c, e: (s, -c, e))(*good(q)))
    assert _composite_error() > 1e-3


def test_dropped_mass_matrix_is_caught(monkeypatch):
    orig = filters.InnerOperator.__call__

    def bad(self, V):
        saved = self.B
        self.B = sp.identity(saved.shape[0], dtype=complex, format="csr")
        try:
            return orig(self, V)
        finally:
            self.B = saved
    monkeypatch.setattr(filters.InnerOperator, "__call__", bad)
    assert _diag_filter_error() > 1e-3


def test_ignored_pivots_are_caught(monkeypatch):
    orig = banded.BandLU.solve

    def bad(self, rhs):
        saved = self.ipiv
        self.ipiv = np.arange(self.n, dtype=np.int32)
        try:
            return orig(self, rhs)
        finally:
            self.ipiv = saved
    monkeypatch.setattr(banded.BandLU, "solve", bad)
    assert _band_error() > 1e-3


def test_wrong_basis_for_ritz_vectors_is_caught(monkeypatch):
    import scipy.linalg as sl

    def bad(A, B, U, sigma):
        V = hsrr.orth(U)
        AV, BV = A @ V, B @ V
        Wm = hsrr.orth(AV - sigma * BV)
        lam, vr = sl.eig(Wm.conj().T @ AV, Wm.conj().T @ BV)
        X = Wm @ vr                                      # W instead of V
        X = X / np.linalg.norm(X, axis=0)
        return X, lam, X
    monkeypatch.setattr(hsrr, "hsrr", bad)
    assert _hsrr_error() > 1e-6
