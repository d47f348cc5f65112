"""Pins of the residual form of the composite filter (the precision form's arithmetic):
it must equal the composite filter applied directly and the simple rule with p q
poles (Thm. Rcrm), for any column shifts, and its correction term must vanish on
exact eigenvectors."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import coeffs, filters, gmres, precision
from paper_2310_18043_amd import workloads as W


def _pencil():
    A, B = W.convdiff_pencil(10, mass=(0.5, 1.5), seed=2)
    lam = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam.real)[40] + 0.05j
    r = W.midgap_radius(lam, c, 8)
    return A, B, c, r, lam


@pytest.mark.parametrize("q", [4, 8, 3])
def test_residual_form_equals_composite_and_simple_rule(q):
    A, B, c, r, _ = _pencil()
    p = 4
    G = filters.InnerOperator(A, B, c, r, p)
    shifts, wts, extra = coeffs.outer_shifts(q)
    X = W.start_block(A.shape[0], 6, 3)
    rng = np.random.default_rng(5)
    lam = c + r * 0.7 * (rng.standard_normal(6) + 1j * rng.standard_normal(6))   # arbitrary shifts
    U_res = precision.composite_filter_residual(A, B, G, X, lam, shifts, wts, extra, tol=1e-14)
    U_dir, _, _, _ = gmres.composite_filter_apply(G, X, shifts, wts, extra, tol=1e-14)
    U_simple = filters.simple_filter(A, B, c, r, p * q, X)
    assert np.linalg.norm(U_res - U_dir) <= 1e-10 * np.linalg.norm(U_dir)
    assert np.linalg.norm(U_res - U_simple) <= 1e-10 * np.linalg.norm(U_simple)


def test_correction_vanishes_on_eigenvectors():
    A, B, c, r, _ = _pencil()
    lam, V = sl.eig(A.toarray(), B.toarray())
    inside = np.argsort(np.abs(lam - c))[:3]
    X = V[:, inside] / np.linalg.norm(V[:, inside], axis=0)
    G = filters.InnerOperator(A, B, c, r, 4)
    shifts, wts, extra = coeffs.outer_shifts(8)
    U = precision.composite_filter_residual(A, B, G, X, lam[inside], shifts, wts, extra)
    # U = X diag(R_{pq}(lambda)) up to the eigenvector residual
    Rv = coeffs.composite_filter(lam[inside], c, r, 4, 8)
    assert np.linalg.norm(U - X * Rv[None, :]) <= 1e-9 * np.linalg.norm(U)


def test_dropping_the_correction_is_caught():
    # the correction term matters for non-eigenvectors: X diag(f(g)) alone is wrong
    A, B, c, r, _ = _pencil()
    G = filters.InnerOperator(A, B, c, r, 4)
    shifts, wts, extra = coeffs.outer_shifts(8)
    X = W.start_block(A.shape[0], 4, 9)
    lam = np.full(4, c)
    U_res = precision.composite_filter_residual(A, B, G, X, lam, shifts, wts, extra)
    fg = coeffs.composite_filter(np.full(4, c), c, r, 4, 8)
    assert np.linalg.norm(U_res - X * fg[None, :]) > 1e-2 * np.linalg.norm(U_res)
