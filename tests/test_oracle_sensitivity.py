"""Pins of the oracle's eigenvalue sensitivities (differentiation form).

The formula d lambda = y^H (dA - lambda dB) x / (y^H B x) is textbook perturbation
theory; these tests fix it against things that do not use it: closed forms for
diagonal pencils, central finite differences of a dense eigensolver on small
random pencils, and the eigenvalue shift of a B = I pencil under A -> A + t I.
"""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import sensitivity as S


def _rand_pencil(n, seed, density=0.6, diag_b=False):
    rng = np.random.default_rng(seed)
    mask = rng.uniform(size=(n, n)) < density
    np.fill_diagonal(mask, True)
    A = np.where(mask, rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), 0)
    if diag_b:
        B = np.diag(rng.uniform(0.5, 1.5, n)).astype(np.complex128)
    else:
        B = np.where(mask, 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))), 0)
        B = B + 3.0 * np.eye(n)
    return sp.csr_matrix(A), sp.csr_matrix(B)


def test_diagonal_pencil_closed_form():
    lam = np.array([1 + 2j, -0.5 + 0.1j, 3.0 - 1j])
    b = np.array([0.7, 1.3, 2.0], dtype=np.complex128)
    A = sp.diags(lam * b, format="csr")
    B = sp.diags(b, format="csr")
    l, X, Y = S.dense_left_right(A, B)
    l, X, Y = S.select(l, X, Y, lam)
    for i in range(3):
        g = np.zeros(3, np.complex128)
        g[i] = 1.0
        gA, gB = S.pencil_vjp(A, B, l, X, Y, g)
        # lambda_i = a_ii / b_ii: d/da_ii = 1/b_ii, d/db_ii = -lambda_i / b_ii
        expA = np.zeros(3, np.complex128); expA[i] = 1 / b[i]
        expB = np.zeros(3, np.complex128); expB[i] = -lam[i] / b[i]
        assert np.allclose(gA, expA, atol=1e-14)
        assert np.allclose(gB, expB, atol=1e-14)


@pytest.mark.parametrize("seed,diag_b", [(1, False), (2, True), (3, False)])
def test_against_central_differences(seed, diag_b):
    n = 7
    A, B = _rand_pencil(n, seed, diag_b=diag_b)
    lam, X, Y = S.dense_left_right(A, B)
    rng = np.random.default_rng(seed + 10)
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    gA, gB = S.pencil_vjp(A, B, lam, X, Y, g)
    h = 1e-6
    for M, grad, which in ((A, gA, "A"), (B, gB, "B")):
        for e in rng.choice(M.nnz, size=min(6, M.nnz), replace=False):
            # a complex entry has two real directions; the eigenvalues are holomorphic
            # in it, so d lambda = derivative * t for a complex step t
            for t in (1.0, 1j):
                Mp = M.copy(); Mp.data[e] += h * t
                Mm = M.copy(); Mm.data[e] -= h * t
                Ap, Bp = (Mp, B) if which == "A" else (A, Mp)
                Am, Bm = (Mm, B) if which == "A" else (A, Mm)
                lp = sl.eigvals(Ap.toarray(), Bp.toarray())
                lm = sl.eigvals(Am.toarray(), Bm.toarray())
                # track each eigenvalue by nearest match
                fd = 0.0
                for i in range(n):
                    jp = np.argmin(np.abs(lp - lam[i]))
                    jm = np.argmin(np.abs(lm - lam[i]))
                    fd += g[i] * (lp[jp] - lm[jm]) / (2 * h)
                assert abs(fd - grad[e] * t) <= 1e-6 * max(1.0, abs(fd)), (which, e, t)


def test_identity_shift_moves_every_eigenvalue_by_one():
    # A -> A + t I with B = I shifts every eigenvalue by t: sum over the diagonal
    # entries of d lambda_i / d A_jj is 1 (trace of the spectral projector)
    A, _ = _rand_pencil(6, 5)
    B = sp.identity(6, dtype=np.complex128, format="csr")
    A = sp.csr_matrix(A + sp.identity(6) * 0)   # diagonal stored
    lam, X, Y = S.dense_left_right(A, B)
    A.sort_indices()
    diag_entries = [e for j in range(6) for e in range(A.indptr[j], A.indptr[j + 1])
                    if A.indices[e] == j]
    for i in range(6):
        g = np.zeros(6, np.complex128); g[i] = 1
        gA, gB = S.pencil_vjp(A, B, lam, X, Y, g)
        assert abs(gA[diag_entries].sum() - 1.0) <= 1e-10
        # and scaling B by (1 + t) scales lambda by 1/(1+t): sum_j B_jj d/dB_jj = -lambda
        assert abs(gB.sum() + lam[i]) <= 1e-10 * max(1, abs(lam[i]))


def test_unconjugated_left_vectors_are_caught():
    # a plausible slip (y^T instead of y^H) must fail the finite-difference pin
    n = 6
    A, B = _rand_pencil(n, 7)
    lam, X, Y = S.dense_left_right(A, B)
    g = np.zeros(n, np.complex128); g[0] = 1
    gA_good, _ = S.pencil_vjp(A, B, lam, X, Y, g)
    gA_bad, _ = S.pencil_vjp(A, B, lam, X, Y.conj(), g)
    h = 1e-6
    e = 0
    Ap = A.copy(); Ap.data[e] += h
    Am = A.copy(); Am.data[e] -= h
    lp = sl.eigvals(Ap.toarray(), B.toarray())
    lm = sl.eigvals(Am.toarray(), B.toarray())
    fd = (lp[np.argmin(np.abs(lp - lam[0]))] - lm[np.argmin(np.abs(lm - lam[0]))]) / (2 * h)
    assert abs(fd - gA_good[e]) <= 1e-6 * max(1, abs(fd))
    assert abs(fd - gA_bad[e]) > 1e-3 * max(1, abs(fd))


def test_sparse_condition_numbers_against_dense():
    import scipy.sparse as sp
    from paper_2310_18043_amd import workloads as W
    v = W.random_vfield(8, 20.0, 2)
    A, B = W.convdiff_pencil(8, 1.0, vfield=v, mass=(0.5, 1.5), seed=3)
    lam, X, Y = S.dense_left_right(A, B)
    kap_dense = (np.linalg.norm(X, axis=0) * np.linalg.norm(Y, axis=0)
                 / np.abs(np.sum(Y.conj() * (B @ X), axis=0)))
    pick = np.argsort(lam.real)[[3, 20, 40]]
    kap, Xs, Ys = S.eig_condition_sparse(A, B, lam[pick])
    assert np.allclose(kap, kap_dense[pick], rtol=1e-6)
    # the vectors are eigenvectors
    for k, i in enumerate(pick):
        r = A @ Xs[:, k] - lam[i] * (B @ Xs[:, k])
        assert np.linalg.norm(r) <= 1e-8 * np.abs(lam[i])
