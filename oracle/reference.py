"""Reference eigenvalues of large pencils (oracle).

Test infrastructure only.

Dense QZ cannot reach the benchmark sizes (N >= 16384), so the eigenvalues of
B^{-1}A nearest a point sigma come from shift-and-invert Arnoldi (ARPACK through
SciPy): the eigenvalues mu of (A - sigma B)^{-1} B of largest modulus give
lambda = sigma + 1/mu.  This is the role the paper gives MATLAB's eigs for its
reference values (Sec. 6); an independent library routine, pinned against dense QZ
on small pencils in tests/test_oracle_reference.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla


def nearest_eigenvalues(A, B, sigma: complex, k: int, tol: float = 1e-13, ncv: int | None = None):
    """The k eigenvalues of A x = lambda B x nearest sigma, sorted by distance."""
    ncv = ncv if ncv is not None else min(A.shape[0] - 1, max(2 * k + 1, k + 64))
    lam = sla.eigs(A.tocsc(), k=k, M=B.tocsc(), sigma=sigma, which="LM",
                   return_eigenvectors=False, ncv=ncv, tol=tol)
    return lam[np.argsort(np.abs(lam - sigma))]


def disk_with_count(lam: np.ndarray, centres, counts):
    """Among candidate centres and counts, the disk whose count-th and (count+1)-th
    nearest eigenvalues are furthest apart relatively: (c, r, count, ratio) with r
    halfway between those two distances.  lam must hold every eigenvalue that can be
    among the count+1 nearest to any candidate centre."""
    best = None
    for c in centres:
        d = np.sort(np.abs(lam - c))
        for s in counts:
            ratio = d[s] / d[s - 1]
            if best is None or ratio > best[3]:
                best = (complex(c), float(0.5 * (d[s - 1] + d[s])), int(s), float(ratio))
    return best


def refine_two_sided(A, B, lam, seed: int = 0, iters: int = 3):
    """Eigenvalues near given approximations, improved by two-sided inverse iteration:
    right and left vectors x, y at each approximation (oracle.sensitivity's sparse
    inverse iteration), then the two-sided Rayleigh quotient y^H A x / y^H B x, whose
    error is second order in the vectors' errors.  Returns (lam, kappa_B, relres) with
    kappa_B = ||x|| ||y|| / |y^H B x| and relres the relative residual of the right
    vector, ||A x - lam B x|| / (||A x|| + |lam| ||B x||)."""
    from . import sensitivity
    kap, X, Y = sensitivity.eig_condition_sparse(A, B, lam, seed=seed, iters=iters)
    AX, BX = A @ X, B @ X
    num = np.einsum("ij,ij->j", Y.conj(), AX)
    den = np.einsum("ij,ij->j", Y.conj(), BX)
    out = num / den
    res = np.linalg.norm(AX - BX * out[None, :], axis=0) / (
        np.linalg.norm(AX, axis=0) + np.abs(out) * np.linalg.norm(BX, axis=0))
    return out, kap, res
