"""Projection step HSRR and the relative eigenpair error (oracle).

Test infrastructure only.

HSRR(A, B, U, sigma) is lines 4-7 of Alg. SIsketch (Sec. 2.1):
  V = orth(U); W = orth(A V - sigma B V);
  generalized Schur form of (W^* A V, W^* B V) by QZ;
  lambda_i = (H_A)_ii / (H_B)_ii;  x_i = V P_R V_R(:, i);  Y = [x_1 .. x_ncol].
orth is a thin Householder QR without rank truncation.  The eigenvectors of
the projected pencil come from LAPACK's generalized eigensolver (QZ followed
by back-substitution on the triangular pencil and back-transformation by
P_R), i.e. exactly the product P_R V_R of the paper, column-normalised to unit
2-norm after mapping through V.

The relative error is eq. rel-error (Sec. 3.2):
  e_i = ||A x_i - B x_i lambda_i||_2 / ((|c| + r) ||B x_i||_2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def orth(U: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(np.asarray(U, dtype=np.complex128), mode="reduced")
    return Q


def hsrr(A, B, U: np.ndarray, sigma: complex):
    """Return (Y, lam, X): Ritz values and unit-norm Ritz vectors (Y = X)."""
    V = orth(U)
    AV = A @ V
    BV = B @ V
    W = orth(AV - sigma * BV)
    Ah = W.conj().T @ AV
    Bh = W.conj().T @ BV
    lam, vr = sl.eig(Ah, Bh, right=True, left=False, homogeneous_eigvals=False)
    X = V @ vr
    X = X / np.linalg.norm(X, axis=0)
    return X, lam, X


def rel_errors(A, B, lam: np.ndarray, X: np.ndarray, c: complex, r: float):
    """e_i of eq. rel-error for every column of X."""
    AX = A @ X
    BX = B @ X
    num = np.linalg.norm(AX - BX * lam[None, :], axis=0)
    den = (abs(c) + r) * np.linalg.norm(BX, axis=0)
    return num / den
