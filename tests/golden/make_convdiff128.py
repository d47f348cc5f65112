"""Write the oracle's eigenpairs of the 128 x 128 convection-diffusion workload.

Runs Alg. composite with the CPU oracle (oracle/solver.py) on the pencil and
disk of ``paper_2310_18043_amd.workloads.convdiff_workload()`` (p = 4, q = 8,
w = 128, start block seed 0) and stores the converged eigenvalues inside the
disk, with their relative errors, in ``convdiff128_eigs.txt``.  Only the oracle
computes the stored values.  Takes tens of minutes on one CPU core.

    OPENBLAS_NUM_THREADS=1 python tests/golden/make_convdiff128.py
"""
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import solver  # noqa: E402
from paper_2310_18043_amd import workloads as W  # noqa: E402


def main():
    wl = W.convdiff_workload()
    Y0 = W.start_block(wl.n, wl.w, wl.seed)
    t0 = time.time()
    res = solver.solve_region(wl.A, wl.B, wl.c, wl.r, wl.p, wl.q, Y0, tau=1e-10,
                              gmres_tol=1e-12, s_expected=wl.s_expected)
    dt = time.time() - t0
    # G applications (vectors): n_col for G(Y) plus one per Arnoldi step per column
    apps = [int(wl.w + it.sum()) for it in res.gmres_iters]
    order = np.argsort(res.lam.real)
    out = os.path.join(HERE, "convdiff128_eigs.txt")
    with open(out, "w") as f:
        f.write("# Oracle (Alg. composite, CPU FP64) eigenvalues inside the disk of the\n")
        f.write(f"# 128x128 convection-diffusion workload: c={wl.c}, r={wl.r!r}, p={wl.p}, "
                f"q={wl.q}, w={wl.w}, seed={wl.seed}\n")
        f.write(f"# sweeps={res.sweeps} converged={res.converged} seconds={dt:.0f} "
                f"gmres_steps_max={[int(i.max()) for i in res.gmres_iters]} "
                f"inner_applications={apps}\n")
        f.write("# re im rel_error\n")
        for k in order:
            f.write(f"{float(res.lam[k].real)!r} {float(res.lam[k].imag)!r} {float(res.err[k])!r}\n")
    print(out, len(res.lam), res.sweeps, res.converged, f"{dt:.0f}s")


if __name__ == "__main__":
    main()
