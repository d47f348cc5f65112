"""Multi-shift GMRES, one Krylov space per column (oracle).

Test infrastructure only.

Sec. 3.2 of Chen & Li solves (G - s_j I) U_j = Ytilde for all q shifts on one
Krylov space per right-hand side, using the shift invariance
K_n(G - s I, y) = K_n(G, y) and (G - s I) V_n = V_{n+1} (H - s I~), where H is
the (n+1) x n Arnoldi Hessenberg matrix and I~ is the n x n identity with a
zero row appended.  Zero initial guess, no restart.

Readings where the paper is silent: the stopping rule is, per column,
max over shifts of ||y - (G - s_j) u_j|| / ||y|| <= tol, checked after every
Arnoldi step; orthogonalisation is classical Gram-Schmidt applied twice.
"""
from __future__ import annotations

import numpy as np


def _lstsq_residual(Hs: np.ndarray, rhs: np.ndarray):
    y, *_ = np.linalg.lstsq(Hs, rhs, rcond=None)
    return y, float(np.linalg.norm(rhs - Hs @ y))


def multishift_gmres(G, Yt: np.ndarray, shifts, tol: float = 1e-12,
                     max_iter: int = 150):
    """Solve (G - s_j I) u_{j,k} = Yt[:, k] for every shift j and column k.

    ``G`` maps an N x m block to an N x m block; all unconverged columns are
    passed to it together, but every column keeps its own Arnoldi basis and
    its own least-squares problems.

    Returns (U, iters, converged): U has shape (q, N, ncol), iters[k] is the
    number of Arnoldi steps (applications of G) used for column k.
    """
    Yt = np.asarray(Yt, dtype=np.complex128)
    N, ncol = Yt.shape
    shifts = np.asarray(shifts, dtype=np.complex128)
    q = len(shifts)
    beta = np.linalg.norm(Yt, axis=0)
    bases = [[Yt[:, k] / beta[k]] if beta[k] > 0 else [] for k in range(ncol)]
    H = [np.zeros((max_iter + 1, max_iter), dtype=np.complex128) for _ in range(ncol)]
    iters = np.zeros(ncol, dtype=np.int64)
    done = beta == 0
    sols = [None] * ncol
    while not done.all():
        active = [k for k in range(ncol) if not done[k]]
        n = int(iters[active[0]])
        Wblk = G(np.stack([bases[k][-1] for k in active], axis=1))
        for a, k in enumerate(active):
            w = Wblk[:, a].copy()
            V = np.stack(bases[k], axis=1)            # N x (n+1)
            for _ in range(2):                        # CGS, twice
                h = V.conj().T @ w
                w -= V @ h
                H[k][: n + 1, n] += h
            hn = np.linalg.norm(w)
            H[k][n + 1, n] = hn
            iters[k] = n + 1
            rhs = np.zeros(n + 2, dtype=np.complex128)
            rhs[0] = beta[k]
            Hn = H[k][: n + 2, : n + 1]
            ys, worst = [], 0.0
            for s in shifts:
                Hs = Hn.copy()
                Hs[: n + 1, : n + 1] -= s * np.eye(n + 1)
                y, res = _lstsq_residual(Hs, rhs)
                ys.append(y)
                worst = max(worst, res / beta[k])
            breakdown = hn <= 1e-14 * np.abs(H[k][: n + 2, : n + 1]).max()
            if worst <= tol or breakdown or n + 1 >= max_iter:
                done[k] = True
                Vn = np.stack(bases[k][: n + 1], axis=1)
                sols[k] = (Vn, ys, worst <= tol or breakdown)
            else:
                bases[k].append(w / hn)
    U = np.zeros((q, N, ncol), dtype=np.complex128)
    converged = np.ones(ncol, dtype=bool)
    for k in range(ncol):
        if sols[k] is None:
            continue
        Vn, ys, ok = sols[k]
        converged[k] = ok
        for j in range(q):
            U[j, :, k] = Vn @ ys[j]
    return U, iters, converged


def composite_filter_apply(G, Y: np.ndarray, shifts, weights, extra: float = 0.0,
                           tol: float = 1e-12, max_iter: int = 150):
    """U = sum_j c'_j (G - s_j I)^{-1} G(Y) (+ extra * G(Y) for odd q).

    eq. linearsolve1abs (Sec. 3.2) with the outer weights of the composite
    rule.  Returns (U, Ytilde, iters, converged).
    """
    Yt = G(Y)
    Us, iters, conv = multishift_gmres(G, Yt, shifts, tol, max_iter)
    U = extra * Yt
    for cj, Uj in zip(weights, Us):
        U = U + cj * Uj
    return U, Yt, iters, conv
