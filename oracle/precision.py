"""Residual form of the composite filter (oracle), the arithmetic behind the
precision form.

Test infrastructure only.

For a block X with one shift l_k per column (any complex numbers away from the
poles), write r_k = A x_k - l_k B x_k.  With K_i = p_i B - A one has
K_i x_k = (p_i - l_k) B x_k - r_k, hence

    K_i^{-1} B x_k = x_k / (p_i - l_k) + K_i^{-1} r_k / (p_i - l_k),
    G x_k = g_k x_k + rho_k,   g_k = sum_i w_i / (p_i - l_k),
                               rho_k = sum_i w_i K_i^{-1} r_k / (p_i - l_k)

(G and w_i, p_i as in eq. linearsolve2), and for every outer shift s_j

    (G - s_j)^{-1} G x_k = g_k / (g_k - s_j) x_k - s_j / (g_k - s_j) (G - s_j)^{-1} rho_k.

So the composite filter U = sum_j c'_j (G - s_j)^{-1} G X + e G X (Thm. Rcrm with the
sign of reading R1, e = 1/q for odd q, else 0) equals

    U = X diag(f(g)) - sum_j c'_j s_j Z_j diag(1/(g - s_j)) + e rho,
    f(g) = sum_j c'_j g / (g - s_j) + e g,   Z_j = (G - s_j)^{-1} rho.

This is exact algebra; the paper does not use it.  Its point: when the shifts are
Ritz values of X, rho is as small as the residual, so rounding in the band solves
and outer solves (which only see rho) is relative to the residual, not to X.
"""
from __future__ import annotations

import numpy as np

from . import gmres


def composite_filter_residual(A, B, G, X: np.ndarray, lam: np.ndarray, shifts, weights,
                              extra: float = 0.0, tol: float = 1e-12, max_iter: int = 150):
    """U by the residual form above; G is an ``filters.InnerOperator`` (its factors,
    poles and weights are used for rho).  Returns U."""
    X = np.asarray(X, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.complex128)
    R = A @ X - (B @ X) * lam[None, :]
    g = np.zeros(X.shape[1], dtype=np.complex128)
    rho = np.zeros_like(X)
    for wi, pi, f in zip(G.weights, G.poles, G.factors):
        d = wi / (pi - lam)
        g = g + d
        rho = rho + f.solve(R) * d[None, :]
    fg = extra * g
    U = extra * rho
    if len(shifts) > 0:
        Zs, _, _ = gmres.multishift_gmres(G, rho, shifts, tol, max_iter)
        for sj, cj, Zj in zip(shifts, weights, Zs):
            fg = fg + cj * g / (g - sj)
            U = U - Zj * (cj * sj / (g - sj))[None, :]
    return U + X * fg[None, :]
