"""Pins of the oracle's projection step and of Alg. composite end to end.

* Rayleigh-Ritz exactness: an exact invariant subspace in gives the exact
  eigenvalues out (HSRR, Sec. 2.1).
* eq. rel-error is zero on exact eigenpairs and invariant under scaling.
* Eigenvalues in closed form: balanced tridiagonal Toeplitz
  a + 2 sqrt(bc) cos(k pi/(n+1)); the literal (non-normal) Toeplitz pencil
  for small n; brute-force dense QZ (LAPACK) on small random-mass
  convection-diffusion pencils.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import hsrr, solver
from paper_2310_18043_amd import workloads as W

RNG = np.random.default_rng(5)


def _match(got, want):
    """Largest distance from each computed eigenvalue to the nearest reference."""
    return np.abs(np.asarray(got)[:, None] - np.asarray(want)[None, :]).min(axis=1).max()


def test_hsrr_exact_on_invariant_subspace():
    n = 80
    lam = RNG.standard_normal(n) + 1j * RNG.standard_normal(n)
    b = RNG.uniform(0.5, 1.5, n)
    A, B = W.diagonal_pencil(lam, b)
    idx = np.array([3, 17, 40, 41, 77])
    E = np.zeros((n, len(idx)), dtype=np.complex128)
    E[idx, np.arange(len(idx))] = 1.0
    U = E @ (RNG.standard_normal((5, 5)) + 1j * RNG.standard_normal((5, 5)))
    _, got, X = hsrr.hsrr(A, B, U, sigma=0.1 + 0.2j)
    assert _match(got, lam[idx]) <= 1e-13
    err = hsrr.rel_errors(A, B, got, X, 0.0, 1.0)
    assert err.max() <= 1e-14
    Xp = X + 1e-3 * (RNG.standard_normal(X.shape) + 1j * RNG.standard_normal(X.shape))
    e1 = hsrr.rel_errors(A, B, got, Xp, 0.0, 1.0)
    e2 = hsrr.rel_errors(A, B, got, Xp * (3 - 4j), 0.0, 1.0)
    assert e1.min() > 1e-6 and np.allclose(e1, e2, rtol=1e-12, atol=0)


def test_rel_error_definition_scale():
    # e = ||A x - B x lam|| / ((|c| + r) ||B x||) on a hand-built 2 x 2 case
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[2.0, 1.0], [0.0, 3.0]], dtype=complex))
    B = sp.identity(2, dtype=complex, format="csr")
    x = np.array([[1.0], [0.0]], dtype=complex)
    e = hsrr.rel_errors(A, B, np.array([2.5 + 0j]), x, 1.0 + 0j, 1.0)
    assert abs(e[0] - 0.5 / 2.0) <= 1e-15


@pytest.mark.slow
def test_solve_region_balanced_toeplitz_closed_form():
    wl = W.toeplitz_workload(n=400, w=32, count=20)
    Y0 = W.start_block(wl.n, wl.w, 0)
    res = solver.solve_region(wl.A, wl.B, wl.c, wl.r, wl.p, wl.q, Y0, s_expected=20)
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    assert res.converged and len(res.lam) == len(inside) == 20
    assert _match(res.lam, inside) <= 1e-13
    assert _match(inside, res.lam) <= 1e-13
    assert res.err.max() <= 1e-10


def test_solve_region_literal_toeplitz_small():
    n = 30
    A, B = W.toeplitz_pencil(n, 0.0, 1.0, W.TOEPLITZ_C, balanced=False)
    exact = W.toeplitz_eigs(n, 0, 1, W.TOEPLITZ_C)
    c = exact[10] + 0.01
    r = W.midgap_radius(exact, c, 4)
    res = solver.solve_region(A, B, c, r, 4, 4, W.start_block(n, 8, 2), s_expected=4)
    inside = exact[np.abs(exact - c) < r]
    assert len(res.lam) == 4
    # non-normal pencil: first-order bound |dlambda| <= kappa * e * (|c| + r)
    w, vl, vr = sl.eig(A.toarray(), B.toarray(), left=True, right=True)
    for lam, e in zip(res.lam, res.err):
        i = np.argmin(np.abs(w - lam))
        x, y = vr[:, i], vl[:, i]
        kappa = np.linalg.norm(x) * np.linalg.norm(y) / abs(y.conj() @ x)
        assert np.abs(inside - lam).min() <= 2 * kappa * e * (abs(c) + r) + 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_solve_region_random_mass_vs_dense_qz(seed):
    n = 14
    A, B = W.convdiff_pencil(n, 1.0, (20.0, 10.0), 0.05j, (0.5, 1.5), seed=seed)
    lam_all = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam_all.real)[60] + 0.05j
    r = W.midgap_radius(lam_all, c, 10)
    res = solver.solve_region(A, B, c, r, 4, 8, W.start_block(n * n, 16, seed),
                              s_expected=10)
    inside = lam_all[np.abs(lam_all - c) < r]
    assert res.converged and len(res.lam) == len(inside) == 10
    assert _match(res.lam, inside) <= 1e-9 * abs(c)
    assert res.err.max() <= 1e-10


def test_solve_region_adaptive_vs_dense_qz():
    # Alg. composite2 on a small random-mass pencil: every pair inside the disk,
    # against dense QZ
    import scipy.linalg as sl
    n = 20
    A, B = W.convdiff_pencil(n, mass=(0.5, 1.5), seed=6)
    lam_all = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam_all.real)[150] + 0.05j
    r = W.midgap_radius(lam_all, c, 12)
    res = solver.solve_region_adaptive(A, B, c, r, 4, 4, 64, W.start_block(n * n, 16, 1),
                                       s_expected=12)
    inside = lam_all[np.abs(lam_all - c) < r]
    assert res.converged and len(res.lam) == len(inside) == 12
    d = np.abs(res.lam[:, None] - inside[None, :]).min(axis=1)
    assert np.all(d <= 1e-11 * np.abs(res.lam)), d.max()
    assert res.err.max() <= 1e-10


def test_solve_region_adaptive_balanced_toeplitz_closed_form():
    wl = W.toeplitz_workload(n=200, w=16, count=8)
    res = solver.solve_region_adaptive(wl.A, wl.B, wl.c, wl.r, 4, 4, 64,
                                       W.start_block(wl.n, 16, 0), s_expected=8)
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    assert res.converged and len(res.lam) == len(inside)
    d = np.abs(res.lam[:, None] - inside[None, :]).min(axis=1)
    assert np.all(d <= 1e-10 * np.abs(inside).max()), d.max()
