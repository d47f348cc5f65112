"""Alg. composite: composite-rule filter inside subspace iteration (oracle).

Test infrastructure only.

Steps (Sec. 3.2, Alg. composite):
  1. poles/weights of the inner p-point rule and the q outer shifts/weights;
  2. pre-factorize K_i = p_i B - A, i = 1..p;
  3. G(V) = sum_i w_i K_i^{-1} B V;
  4. Y = orth(random N x n_col);
  5. repeat: Ytilde = G(Y); U_j = (G - s_j I)^{-1} Ytilde by multi-shift
     GMRES; U = sum_j c'_j U_j; [Y, Lambda, X] = HSRR(A, B, U, sigma);
     count the filtered pairs (inside D and e_i < tau_g)
     until the count is unchanged and every filtered e_i <= tau.

Readings where the paper leaves room (Sec. 3.2 and Sec. 6):
  * "inside D" is strict, |lambda - c| < r;
  * the count starts undefined, so at least two sweeps run unless the first
    sweep already finds the expected number of pairs all below tau (the
    paper stops after the first sweep in that case, Sec. 6.3);
  * at most ``max_it`` sweeps (10 in Sec. 6.3);
  * sigma defaults to c (Sec. 6).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import coeffs, filters, gmres, hsrr


@dataclasses.dataclass
class SolveResult:
    lam: np.ndarray          # filtered eigenvalues inside D
    X: np.ndarray            # their unit-norm right vectors (N x count)
    err: np.ndarray          # their relative errors e_i
    all_lam: np.ndarray      # every Ritz value of the last sweep
    all_err: np.ndarray
    sweeps: int
    gmres_iters: list        # per sweep: per-column Arnoldi step counts
    converged: bool


def solve_region(A, B, c: complex, r: float, p: int, q: int, Y0: np.ndarray,
                 tau: float = 1e-10, tau_g: float = 1e-2, sigma=None,
                 gmres_tol: float = 1e-12, max_it: int = 10,
                 s_expected=None, gmres_max_iter: int = 150) -> SolveResult:
    A = A.tocsr(); B = B.tocsr()
    sigma = complex(c) if sigma is None else complex(sigma)
    G = filters.InnerOperator(A, B, c, r, p)
    shifts, wts, extra = coeffs.outer_shifts(q)
    Y = hsrr.orth(Y0)
    prev = None
    its = []
    lam = X = err = None
    converged = False
    for t in range(1, max_it + 1):
        U, _, it, _ = gmres.composite_filter_apply(G, Y, shifts, wts, extra,
                                                   gmres_tol, gmres_max_iter)
        its.append(it)
        Y, lam, X = hsrr.hsrr(A, B, U, sigma)
        err = hsrr.rel_errors(A, B, lam, X, c, r)
        inside = np.abs(lam - c) < r
        filt = inside & (err < tau_g)
        count = int(filt.sum())
        all_small = bool(np.all(err[filt] <= tau))
        if all_small and (count == prev or (t == 1 and s_expected is not None
                                            and count == s_expected)):
            converged = True
            break
        prev = count
    filt = (np.abs(lam - c) < r) & (err < tau_g)
    return SolveResult(lam[filt], X[:, filt], err[filt], lam, err, t, its,
                       converged)
