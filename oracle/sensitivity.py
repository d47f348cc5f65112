"""First-order eigenvalue sensitivities of the pencil (oracle).

Test infrastructure only.

The paper does not differentiate its eigenvalues; the differentiation form uses
textbook first-order perturbation theory.  For a simple eigenvalue lambda of
A x = lambda B x with right vector x and left vector y (y^H A = lambda y^H B):

    d lambda = y^H (dA - lambda dB) x / (y^H B x),

so for a stored entry A[j, k] the partial derivative is conj(y_j) x_k / (y^H B x) and
for B[j, k] it is -lambda conj(y_j) x_k / (y^H B x).  The left vectors are the right
eigenvectors of the adjoint pencil (A^H, B^H) at conj(lambda).

Here x and y come from one dense generalized eigen-decomposition (LAPACK through
SciPy), so this oracle is for small pencils.  ``pencil_vjp`` is the contraction
sum_i g_i d lambda_i / d (stored entry), written entry by entry.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp


def dense_left_right(A, B):
    """All eigenvalues with right vectors X and left vectors Y (columns), dense."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    lam, Y, X = sl.eig(Ad, Bd, left=True, right=True)
    return lam, X, Y


def select(lam, X, Y, targets):
    """The dense eigenpairs nearest to ``targets`` (one each, distinct)."""
    idx = []
    for t in np.asarray(targets):
        j = int(np.argmin(np.abs(lam - t)))
        if j in idx:
            raise ValueError("two targets select the same eigenvalue")
        idx.append(j)
    idx = np.array(idx, dtype=int)
    return lam[idx], X[:, idx], Y[:, idx]


def pencil_vjp(A, B, lam, X, Y, g):
    """(gA, gB): sum_i g_i d lambda_i / d M[j, k] at every stored entry of A and B,
    in CSR order (sorted indices)."""
    A = sp.csr_matrix(A); A.sort_indices()
    B = sp.csr_matrix(B); B.sort_indices()
    lam = np.asarray(lam, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    den = np.array([Y[:, i].conj() @ (B @ X[:, i]) for i in range(len(lam))])

    def contract(M, coef):
        out = np.zeros(M.nnz, dtype=np.complex128)
        for j in range(M.shape[0]):
            for e in range(M.indptr[j], M.indptr[j + 1]):
                k = M.indices[e]
                out[e] = np.sum(coef * Y[j, :].conj() * X[k, :])
        return out

    gA = contract(A, g / den)
    gB = contract(B, -g * lam / den)
    return gA, gB


def eig_condition_sparse(A, B, lam, seed: int = 0, iters: int = 3):
    """Right and left eigenvectors at given (accurate) eigenvalues of a sparse pencil by
    inverse iteration with a sparse LU of A - lambda B (SuperLU through SciPy), and the
    condition numbers kappa_B = ||x|| ||y|| / |y^H B x|.

    kappa_B is the first-order bound |d lambda| <= kappa_B ||dA x - lambda dB x|| / ||x||,
    so an approximate pair with residual norm ||A x - lambda B x|| (unit x) has an
    eigenvalue error of at most kappa_B times that norm, to first order.
    Returns (kappa, X, Y)."""
    import scipy.sparse.linalg as sla
    A = sp.csc_matrix(A)
    B = sp.csc_matrix(B)
    n = A.shape[0]
    rng = np.random.default_rng(seed)
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    X = np.zeros((n, len(lam)), dtype=np.complex128)
    Y = np.zeros_like(X)
    kap = np.zeros(len(lam))
    for k, l in enumerate(lam):
        M = (A - l * B).tocsc()
        lu = sla.splu(M)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        BH = B.conj().T
        for _ in range(iters):
            x = lu.solve(B @ x)
            x /= np.linalg.norm(x)
            y = lu.solve(BH @ y, trans="H")
            y /= np.linalg.norm(y)
        X[:, k], Y[:, k] = x, y
        kap[k] = 1.0 / abs(np.vdot(y, B @ x))
    return kap, X, Y
