"""Write the disks and oracle references of the batched workload: 64 disks on the
256 x 256 random-velocity pencil of workloads.convdiff256_workload.

1. Requested eigenvalue counts log-uniform over [10, 200] (PCG64 seed 4).  (On this
   pencil the eigenvalues fill a thin strip along the real axis with a nearly constant
   density of 0.073 per unit of Re, so a count range of 20x needs a radius range of
   20x; the counts are drawn, the radii follow.)
2. Every eigenvalue of the strip's low end, by shift-invert Arnoldi in overlapping
   windows (oracle.reference.nearest_eigenvalues, 400 eigenvalues each, centres 2000,
   6000, 10000, ..., overlapping), merged.
3. Adjacent disks along the real axis from Re = 0 (workloads.strip_disks: rims in the
   widest relative gaps, counts within +-3 of the request), block width the smallest
   power of two >= 1.25 x count.
4. Each disk's eigenvalues refined by two-sided inverse iteration with kappa_B
   (oracle.reference.refine_two_sided), in 8 processes.

Writes convdiff256_disks.txt (disk, Re c, Im c, r, count, w) and
convdiff256_disk_eigs.txt (disk, Re, Im, kappa_B, relative residual).  Only the
oracle computes the stored eigenvalues.  About an hour on 8 cores.

    python tests/golden/make_convdiff256_batch.py
"""
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "2")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

NDISKS = 64
NPROC = 8


def _window(sigma):
    from oracle import reference
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    lam = reference.nearest_eigenvalues(wl.A, wl.B, sigma, 400, ncv=900)
    return sigma, lam


def _refine(lam):
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    from oracle import reference
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    return reference.refine_two_sided(wl.A, wl.B, lam)


def main():
    import multiprocessing as mp
    from paper_2310_18043_amd import workloads as W
    t0 = time.time()
    rng = np.random.Generator(np.random.PCG64(4))
    want = np.rint(np.exp(rng.uniform(np.log(10), np.log(200), size=NDISKS))).astype(int)
    need = int(want.sum() * 1.15) + 400
    ctx = mp.get_context("spawn")
    found, covered = [], 0.0
    with ctx.Pool(4) as pool:
        # centres 4000 apart: each window reaches about 2450 on either side, so
        # consecutive windows overlap by about 900 along the strip
        top = need / 0.073 + 4000.0
        sig = [2000.0 + 4000.0 * j for j in range(int(np.ceil((top - 2000.0) / 4000.0)) + 1)]
        for sigma, lam in pool.imap(_window, sig):
            d = np.abs(lam - sigma)
            # every eigenvalue within the window's 400th distance is found
            found.append((sigma, d.max(), lam))
            print(f"window {sigma:.0f}: reach {d.max():.0f}, {time.time() - t0:.0f}s", flush=True)
    # merge: keep eigenvalues once, and only up to the first Re beyond which a window
    # boundary might have missed some (consecutive windows must overlap)
    found.sort(key=lambda t: t[0])
    allv = np.concatenate([f[2] for f in found])
    allv = allv[np.argsort(allv.real)]
    keep = [allv[0]]
    for v in allv[1:]:
        if abs(v - keep[-1]) > 1e-8 * abs(v):
            keep.append(v)
    lam = np.array(keep)
    limit = found[0][0] + found[0][1]
    for (s0, r0, _), (s1, r1, _) in zip(found[:-1], found[1:]):
        if s1 - r1 > s0 + r0 - 50.0:                    # gap between windows: stop before it
            limit = min(limit, s0 + r0 - 50.0)
            break
        limit = s1 + r1
    lam = lam[lam.real < limit - 50.0]
    print(f"merged {len(lam)} eigenvalues below Re {limit:.0f}; requested total {want.sum()}", flush=True)
    disks = W.strip_disks(lam, list(want), start=0.0)
    right = disks[-1][0].real + disks[-1][1]
    assert right < lam.real.max(), (right, lam.real.max())
    rows, groups = [], []
    for d, (c, r, s) in enumerate(disks):
        inside = lam[np.abs(lam - c) < r]
        assert len(inside) == s
        w = 16
        while w < 1.25 * s:
            w *= 2
        rows.append((d, c.real, c.imag, r, s, w))
        groups.append(inside)
    with open(os.path.join(HERE, "convdiff256_disks.txt"), "w") as f:
        f.write("# 64 disks along the real axis of the 256x256 random-velocity pencil "
                "(tests/golden/make_convdiff256_batch.py)\n# disk re_c im_c r count w\n")
        for row in rows:
            f.write(f"{row[0]} {row[1]!r} {row[2]!r} {row[3]!r} {row[4]} {row[5]}\n")
    print(f"disks: counts {min(r[4] for r in rows)}..{max(r[4] for r in rows)}, total "
          f"{sum(r[4] for r in rows)}, right edge {right:.0f}, {time.time() - t0:.0f}s", flush=True)
    flat = np.concatenate(groups)
    owner = np.concatenate([np.full(len(g), d) for d, g in enumerate(groups)])
    parts = np.array_split(np.arange(len(flat)), NPROC * 4)
    with ctx.Pool(NPROC) as pool:
        outs = pool.map(_refine, [flat[p_] for p_ in parts])
    ref = np.concatenate([o[0] for o in outs])
    kap = np.concatenate([o[1] for o in outs])
    res = np.concatenate([o[2] for o in outs])
    with open(os.path.join(HERE, "convdiff256_disk_eigs.txt"), "w") as f:
        f.write("# eigenvalues of the 64 disks of convdiff256_disks.txt (ARPACK windows refined by "
                "two-sided inverse iteration)\n# disk re im kappa_B relres\n")
        for d, v, k, e in zip(owner, ref, kap, res):
            f.write(f"{int(d)} {float(v.real)!r} {float(v.imag)!r} {float(k)!r} {float(e)!r}\n")
    print(f"refined {len(ref)}: max relres {res.max():.1e}, kappa {kap.min():.2f}..{kap.max():.2f}, "
          f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
