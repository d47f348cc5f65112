"""Write convdiff128_cond.txt: the eigenvalue condition numbers
kappa_B = ||x|| ||y|| / |y^H B x| of the 100 eigenvalues in convdiff128_eigs.txt,
from the oracle's sparse inverse iteration (oracle.sensitivity.eig_condition_sparse).
They turn residual norms into eigenvalue error bounds (first order):
|lambda_hat - lambda| <= kappa_B ||A x_hat - lambda_hat B x_hat|| for unit x_hat.

Run from the repository root: python tests/golden/make_convdiff128_cond.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sensitivity  # noqa: E402
from paper_2310_18043_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    rows = [[float(x) for x in l.split()] for l in open(os.path.join(HERE, "convdiff128_eigs.txt"))
            if l.strip() and not l.startswith("#")]
    lam = np.array([r[0] + 1j * r[1] for r in rows])
    wl = W.convdiff_workload()
    kap, _, _ = sensitivity.eig_condition_sparse(wl.A, wl.B, lam)
    with open(os.path.join(HERE, "convdiff128_cond.txt"), "w") as f:
        f.write("# kappa_B of the eigenvalues of convdiff128_eigs.txt (same order): re im kappa_B\n")
        f.write("# written by tests/golden/make_convdiff128_cond.py (oracle sparse inverse iteration)\n")
        for l, k in zip(lam, kap):
            f.write(f"{float(l.real)!r} {float(l.imag)!r} {float(k)!r}\n")


if __name__ == "__main__":
    main()
