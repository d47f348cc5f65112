"""Plain, slow, obviously-correct CPU oracle for the composite-rule filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it.

Everything is complex FP64.  Each function cites the passage of Chen & Li,
"Interior Eigensolver Based on Rational Filter with Composite Rule"
(arXiv 2310.18043) that it writes out:

* ``coeffs``   -- trapezoidal poles/weights (eq. pwtp, Sec. 2.2), the
                  composite outer shifts and weights (eq. Rcrm_, Sec. 3.1 and
                  Thm. Rcrm, Sec. 5), the compact form (Lemma compact, Sec. 4.3).
* ``banded``   -- band LU with partial pivoting and the band solves (plain C,
                  ``oracle/csrc/band.c``): the "pre-factorize K_i" step of
                  Alg. composite (Sec. 3.2).
* ``filters``  -- the simple-rule filter R_{c,r,k}(B^{-1}A)Y (eq.
                  discretizedCIoperator) and the inner operator G (eq.
                  linearsolve2).
* ``gmres``    -- per-column multi-shift GMRES (Sec. 3.2, shift invariance of
                  the Krylov space).
* ``hsrr``     -- the projection step HSRR (Sec. 2.1, Alg. SIsketch) and the
                  relative eigenpair error (eq. rel-error).
* ``solver``   -- Alg. composite (Sec. 3.2) around the pieces above, and
                  Alg. composite2 (Sec. 3.2) by the composite identity.
* ``precision``   -- the residual form of the composite filter used by the
                  precision form (exact algebra; not in the paper).
* ``sensitivity`` -- first-order eigenvalue perturbation with dense left/right
                  vectors, and eigenvalue condition numbers by sparse inverse
                  iteration (textbook; not in the paper).

Readings of passages that are ambiguous or in error in the paper:

* Sign of the outer weights: the statement of eq. Rcrm_ pairs
  c_i = -(1/k2) sigma_i/(1+sigma_i) with (R - s_i)^{-1} R, which sums to
  -R_{c,r,k}; the last line of the proof of Thm. Rcrm pairs the same c_i with
  (s_i - R)^{-1} R.  We use c'_j = +(1/q) sigma_j/(1+sigma_j) with
  (G - s_j I)^{-1} G, which equals +R_{c,r,pq}.
* Odd q: the extra term is (1/q) R_{c,r,p}(z) (statement), not 1/p (proof).
* Hessenberg shape in the shift-invariance relation: (n+1) x n.
"""
