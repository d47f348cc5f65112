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


def solve_region_adaptive(A, B, c: complex, r: float, p: int, q: int, q_max: int,
                          Y0: np.ndarray, tau: float = 1e-10, tau_g: float = 1e-2,
                          sigma=None, s_expected=None) -> SolveResult:
    """Alg. composite2 (Sec. 3.2): no subspace iteration; the outer node count k2
    doubles from q while the block stays Y = orth(Y0).

    At level k2 the algorithm forms U = sum_j c_j^{(k2)} (G - s_j^{(k2)} I)^{-1} G(Y)
    over all k2 outer nodes.  (The shortcut of reusing the k2 solutions and adding
    only the new nodes relies on s^{(k2)} being a subset of s^{(2 k2)}, which does not
    hold for the nodes theta_j = (2j - 1) pi / k2; every node is re-solved.)  By the
    composite identity that sum equals the simple-rule filter with p k2 poles applied
    to Y, which is what this oracle computes, with direct band solves.  Then HSRR,
    the ghost test, and the same stopping rule as Alg. composite (the level plays the
    role of the sweep).  Levels stop at q_max.
    """
    A = A.tocsr(); B = B.tocsr()
    sigma = complex(c) if sigma is None else complex(sigma)
    Y = hsrr.orth(Y0)
    prev = None
    lam = X = err = None
    converged = False
    levels = 0
    k2 = q
    while k2 <= q_max:
        levels += 1
        U = filters.simple_filter(A, B, c, r, p * k2, Y)
        _, lam, X = hsrr.hsrr(A, B, U, sigma)
        err = hsrr.rel_errors(A, B, lam, X, c, r)
        inside = np.abs(lam - c) < r
        filt = inside & (err < tau_g)
        count = int(filt.sum())
        all_small = bool(np.all(err[filt] <= tau))
        if all_small and (count == prev or (levels == 1 and s_expected is not None
                                            and count == s_expected)):
            converged = True
            break
        prev = count
        k2 *= 2
    filt = (np.abs(lam - c) < r) & (err < tau_g)
    return SolveResult(lam[filt], X[:, filt], err[filt], lam, err, levels, [], converged)
