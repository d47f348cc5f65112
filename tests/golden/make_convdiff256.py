"""Write the oracle's references for the 256 x 256 random-velocity workload
(workloads.convdiff256_workload: N = 65536, bandwidth 256, p = q = 8, w = 256).

1. The 400 eigenvalues nearest 2000 by shift-invert Arnoldi
   (oracle.reference.nearest_eigenvalues) and the disk recipe of
   workloads.CONVDIFF256_DISK, checked to reproduce the stored disk.
2. The eigenvalues inside the disk, refined by two-sided inverse iteration with
   their condition numbers kappa_B (oracle.reference.refine_two_sided), into
   convdiff256_eigs.txt.
3. Sketches (128 Gaussian vectors, seed 1234) and exact column norms of
   G(X) = sum_i w_i K_i^{-1} B X (the simple rule with p = 8 poles) on
   X = start_block(N, 256, seed 11), and of the filter R_{c,r,pq}(B^{-1}A) Y (the
   simple rule with pq = 64 poles, Thm. Rcrm) on Y = start_block(N, 256, seed 0),
   into convdiff256_sketch.npz.  The terms of each rule are formed in 8 processes
   (oracle.filters.simple_filter_terms) and added in pole order.

Only the oracle computes the stored values.  About an hour on 8 cores, 20 GB.

    python tests/golden/make_convdiff256.py
"""
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

SKETCH_SEED = 1234
NPROC = 8


def _terms(args):
    k, idx, seed, width = args
    from oracle import filters
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    Y = W.start_block(wl.n, width, seed)
    return filters.simple_filter_terms(wl.A, wl.B, wl.c, wl.r, k, Y, idx)


def _refine(args):
    lam = args
    from oracle import reference
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    return reference.refine_two_sided(wl.A, wl.B, lam)


def _rule(pool, k, seed, width):
    chunks = [list(range(j, k, NPROC)) for j in range(NPROC)]
    parts = pool.map(_terms, [(k, c, seed, width) for c in chunks])
    # add the poles' terms in pole order: term i is in chunk i % NPROC
    return sum(parts[1:], parts[0])


def main():
    import multiprocessing as mp
    from oracle import reference
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    t0 = time.time()
    lam = reference.nearest_eigenvalues(wl.A, wl.B, 2000.0, 400, ncv=900)
    Rmax = np.abs(lam - 2000.0).max()
    best = None
    for cx in np.arange(1200.0, 2800.0, 5.0):
        for cy in np.arange(-6.0, 6.1, 1.0):
            c = complex(cx, cy)
            d = np.sort(np.abs(lam - c))
            for s in range(185, 216):
                ratio = d[s] / d[s - 1]
                r = 0.5 * (d[s - 1] + d[s])
                if abs(c - 2000.0) + 1.2 * r > Rmax:
                    continue
                if best is None or ratio > best[3]:
                    best = (c, r, s, ratio)
    c, r, s, _ = best
    print("disk", best, f"{time.time() - t0:.0f}s", flush=True)
    assert abs(c - wl.c) < 1e-9 and abs(r - wl.r) < 1e-6 * r and s == wl.s_expected, best
    inside = lam[np.abs(lam - c) < r]
    ctx = mp.get_context("spawn")
    with ctx.Pool(NPROC) as pool:
        parts = pool.map(_refine, np.array_split(inside, NPROC))
        lam_ref = np.concatenate([p_[0] for p_ in parts])
        kap = np.concatenate([p_[1] for p_ in parts])
        res = np.concatenate([p_[2] for p_ in parts])
        print("refined", len(lam_ref), "max relres", res.max(), "kappa range", kap.min(), kap.max(),
              f"{time.time() - t0:.0f}s", flush=True)
        order = np.argsort(lam_ref.real)
        with open(os.path.join(HERE, "convdiff256_eigs.txt"), "w") as f:
            f.write("# eigenvalues of the 256x256 random-velocity workload inside its disk "
                    f"c={wl.c}, r={wl.r!r} (ARPACK near 2000, refined by two-sided inverse iteration)\n")
            f.write("# written by tests/golden/make_convdiff256.py: re im kappa_B relres\n")
            for k in order:
                f.write(f"{float(lam_ref[k].real)!r} {float(lam_ref[k].imag)!r} {float(kap[k])!r} "
                        f"{float(res[k])!r}\n")
        S = W.start_block(wl.n, 128, SKETCH_SEED)
        G = _rule(pool, wl.p, 11, wl.w)
        print("G", f"{time.time() - t0:.0f}s", flush=True)
        U = _rule(pool, wl.p * wl.q, wl.seed, wl.w)
        print("filter", f"{time.time() - t0:.0f}s", flush=True)
    np.savez(os.path.join(HERE, "convdiff256_sketch.npz"), sketch_seed=SKETCH_SEED,
             g_sketch=S.conj().T @ G, g_norms=np.linalg.norm(G, axis=0), g_seed=11,
             f_sketch=S.conj().T @ U, f_norms=np.linalg.norm(U, axis=0), f_seed=wl.seed,
             k=wl.p * wl.q, c=wl.c, r=wl.r)
    print("done", f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
