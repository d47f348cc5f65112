"""Rational filters applied to a block of vectors (oracle).

Test infrastructure only.

* ``simple_filter``  -- R_{c,r,k}(B^{-1}A) Y = sum_{i=1}^k w_i (p_i B - A)^{-1} B Y,
  eq. discretizedCIoperator with the trapezoidal poles/weights of eq. pwtp
  (Sec. 2.2).  With k = p q this is the exact value the composite method
  reaches once its outer solves have converged (Thm. Rcrm, Sec. 5).
* ``InnerOperator``  -- G(V) = sum_{i=1}^{p} w_i K_i^{-1} B V with
  K_i = p_i B - A pre-factorized (eq. linearsolve2; Alg. composite, Sec. 3.2).
"""
from __future__ import annotations

import numpy as np

from . import banded, coeffs


def pencil_bandwidths(A, B):
    """Band extents of pattern(A) union pattern(B)."""
    kla, kua = banded.bandwidths(A)
    klb, kub = banded.bandwidths(B)
    return max(kla, klb), max(kua, kub)


class InnerOperator:
    """G(V) = sum_i w_i (p_i B - A)^{-1} B V for the p-point trapezoidal rule."""

    def __init__(self, A, B, c: complex, r: float, p: int):
        self.A, self.B = A.tocsr(), B.tocsr()
        self.poles, self.weights = coeffs.trapezoid_nodes(c, r, p)
        kl, ku = pencil_bandwidths(A, B)
        self.factors = []
        for pi in self.poles:
            f = banded.band_lu(pi * self.B - self.A, kl, ku)
            if f.info != 0:
                raise ZeroDivisionError(f"exact zero pivot at pole {pi}")
            self.factors.append(f)
        self.applications = 0      # number of vectors G has been applied to

    def __call__(self, V: np.ndarray) -> np.ndarray:
        V = np.asarray(V, dtype=np.complex128)
        BV = self.B @ V
        out = np.zeros_like(BV)
        for wi, f in zip(self.weights, self.factors):
            out = out + wi * f.solve(BV)
        self.applications += 1 if V.ndim == 1 else V.shape[1]
        return out


def simple_filter(A, B, c: complex, r: float, k: int, Y: np.ndarray) -> np.ndarray:
    """R_{c,r,k}(B^{-1}A) Y by k independent direct band solves."""
    return InnerOperator(A, B, c, r, k)(Y)


def simple_filter_terms(A, B, c: complex, r: float, k: int, Y: np.ndarray, indices) -> np.ndarray:
    """The terms i in ``indices`` of the simple rule, sum_i w_i (p_i B - A)^{-1} B Y,
    summed in the given order (the poles one at a time, so that the k terms can be
    formed in separate processes and added afterwards)."""
    A, B = A.tocsr(), B.tocsr()
    poles, weights = coeffs.trapezoid_nodes(c, r, k)
    kl, ku = pencil_bandwidths(A, B)
    BY = B @ np.asarray(Y, dtype=np.complex128)
    out = np.zeros_like(BY)
    for i in indices:
        f = banded.band_lu(poles[i] * B - A, kl, ku)
        if f.info != 0:
            raise ZeroDivisionError(f"exact zero pivot at pole {poles[i]}")
        out = out + weights[i] * f.solve(BY)
    return out
