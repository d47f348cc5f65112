"""Autotuner for the launch shapes of the solver.

For a workload (pencil shape, p, q, w, precision) it times the whole hot path --
rf_factor_shifts + rf_solve_region on the device -- for every combination of

* tile      the band tile nb (the smallest power of two >= the bandwidth, and twice it
            when that is still <= 256),
* trsm_cols right-hand sides per band-solve workgroup (1, 2, 4; also 8 at tile 256),
* subblock  the Krylov sub-block width b (16, 32, dividing w),

keeps the fastest combination whose run converged with the expected count, and
records it in ``tuned.json`` beside this file, keyed by the shape.  ``Plan`` reads
the table: a key that matches the plan's shape fills the options the caller left
automatic (0).

    python -m paper_2310_18043_amd.tune convdiff128 convdiff256 --write
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned.json")


def shape_key(n: int, kl: int, ku: int, p: int, q: int, w: int, precision: int) -> str:
    return f"n={n},kl={kl},ku={ku},p={p},q={q},w={w},precision={precision}"


def bandwidths(A, B):
    def bw(M):
        M = M.tocoo()
        d = M.row - M.col
        return (int(d.max()) if d.size else 0), (int((-d).max()) if d.size else 0)
    kla, kua = bw(A)
    klb, kub = bw(B)
    return max(kla, klb), max(kua, kub)


def load_table() -> dict:
    if not os.path.exists(TABLE):
        return {}
    with open(TABLE) as f:
        return json.load(f)


def lookup(A, B, p: int, q: int, w: int, precision: int):
    """The tuned options for this shape, or None."""
    kl, ku = bandwidths(A, B)
    return load_table().get(shape_key(A.shape[0], kl, ku, p, q, w, precision))


def _workloads():
    from paper_2310_18043_amd import workloads as W
    return {
        "convdiff128": (lambda: W.convdiff_workload(), {}),
        "convdiff256": (lambda: W.convdiff256_workload(), {"max_krylov_blocks": 60}),
        "randv128": (lambda: W.random_velocity_workload(), {"max_krylov_blocks": 60}),
    }


def tune(name: str, precision: int = 0, reps: int = 1, log=print):
    import numpy as np
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    make, extra = _workloads()[name]
    wl = make()
    kl, ku = bandwidths(wl.A, wl.B)
    nb0 = 16
    while nb0 < max(kl, ku):
        nb0 *= 2
    tiles = [nb0] + ([2 * nb0] if 2 * nb0 <= 256 else [])
    Y0 = torch.from_numpy(W.start_block(wl.n, wl.w, wl.seed)).cuda()
    rows = []
    for tile in tiles:
        for cw in ((1, 2, 4, 8) if tile == 256 else (1, 2, 4)):
            for b in (16, 32):
                if wl.w % b:
                    continue
                P = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w, tuned=False,
                               expected_count=wl.s_expected, tile=tile, trsm_cols=cw, subblock=b,
                               precision=precision, **extra)
                P.factor_shifts()
                res = P.solve_region(Y0, allow_noconv=True)          # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    P.factor_shifts()
                    res = P.solve_region(Y0, allow_noconv=True)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1000.0 / reps
                good = int(np.sum((np.abs(res["lam"] - wl.c) < wl.r) & (res["err"] <= 1e-10)))
                ok = res["converged"] and good == wl.s_expected
                rows.append({"tile": tile, "trsm_cols": cw, "subblock": b, "ms": round(ms, 3),
                             "converged": bool(ok), "sweeps": res["sweeps"]})
                log(f"[tune] {name} precision={precision} tile={tile} cw={cw} b={b}: {ms:.1f} ms "
                    f"{'ok' if ok else 'NOT CONVERGED'}")
                P.close()
                del P
                torch.cuda.empty_cache()
    good_rows = [r for r in rows if r["converged"]]
    if not good_rows:
        raise RuntimeError(f"no converged configuration for {name}")
    best = min(good_rows, key=lambda r: r["ms"])
    key = shape_key(wl.n, kl, ku, wl.p, wl.q, wl.w, precision)
    return key, {"workload": name, "tile": best["tile"], "trsm_cols": best["trsm_cols"],
                 "subblock": best["subblock"], "ms": best["ms"], "candidates": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--precision", type=int, nargs="+", default=[0])
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--write", action="store_true", help="merge the results into tuned.json")
    ap.add_argument("--out", default=None, help="also write the results to this JSON file")
    args = ap.parse_args(argv)
    table = load_table()
    found = {}
    for name in args.workloads:
        for prec in args.precision:
            key, entry = tune(name, prec, args.reps, log=lambda m: print(m, flush=True))
            found[key] = entry
            print(f"[tune] {key}: {entry['tile']}/{entry['trsm_cols']}/{entry['subblock']} "
                  f"{entry['ms']} ms", flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(found, f, indent=1)
    if args.write:
        table.update(found)
        with open(TABLE, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    sys.exit(main())
