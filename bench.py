"""Benchmark of the composite-rule interior eigensolver on one MI355X.

One step = the whole hot path on one workload: rf_factor_shifts (band LU of
the p shifted pencils) + rf_solve_region (Alg. composite: composite filter by
block multi-shift GMRES, HSRR, ghost test, until converged).  The workload is
the 128 x 128 upwind convection-diffusion pencil (N = 16384, bandwidth 128,
D = 1, v = (20, 10), +0.05i, B = diag U[0.5, 1.5]), ~100 eigenvalues in the
disk, p = 4, q = 8, block width 128, complex FP64.  Inputs are resident on the
device before the timed region.

Prints ONE JSON line:
  value        converged eigenpairs (inside D, e <= 1e-10) per second
  roofline     the band-solve kernel (the inner operator G, the dominant kernel):
               algorithmic FP64 flops per launch / HIP-event-timed duration
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
  filter_apply one composite filter application: algorithmic GB/s and % of peak

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and matrix) peak
PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector peak (complex64 band solves)
# stored HBM traffic of the band-solve kernel that the headline plan runs (rocprofv3 passes)
TRAFFIC_FILES = {
    "band_solve_cluster_kernel": os.path.join(HERE, "profiles", "band_solve_cluster_convdiff128_traffic.json"),
    "band_solve_kernel": os.path.join(HERE, "profiles", "band_solve_convdiff128_traffic.json"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def solve_flops_per_column(n, kl, ku, p):
    """Band-exact flops of sum_i w_i K_i^{-1} for one right-hand side.

    Forward sweep with L (kl multipliers per column) and backward sweep with
    U (kl + ku super-diagonals), 8 real flops per complex multiply-add, for
    each of the p poles.
    """
    return 8.0 * p * n * (2 * kl + ku)


def solve_bytes_per_launch(n, kl, ku, p, cols):
    """Algorithmic HBM bytes of one band-solve launch: every factor once
    (LAPACK band size (2kl+ku+1) n complex + n pivots per pole), the
    right-hand sides read once, the p weighted solutions written once."""
    factor = p * ((2 * kl + ku + 1) * n * 16 + 4 * n)
    return factor + cols * n * 16 * (1 + p)


def host_cpu():
    """(model name, logical CPUs available to this process)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


def _oracle_pole_term(args):
    """One pole's term w_i K_i^{-1} B X of the oracle's inner operator (a worker of the
    all-cores CPU baseline)."""
    name, idx, seed, width = args
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    from oracle import filters
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff_workload()
    X = W.start_block(wl.n, width, seed)
    return filters.simple_filter_terms(wl.A, wl.B, wl.c, wl.r, wl.p, X, idx)


def cpu_baseline(wl, cols_per_step):
    """Time the CPU oracle on a bounded sample of the workload and scale it to
    eigenpairs/s.

    Sample: the oracle's inner operator (its plain-C band LU of all p shifted
    pencils) and one application of G to the whole w-column start block (p band
    solves per column).  The full step is estimated as the p factorizations plus
    the number of columns G was applied to in one GPU step, at the sampled
    per-column cost; the oracle's orthogonalisation, least squares and projection
    are left out, which favours the CPU.
    """
    from oracle import filters
    t0 = time.time()
    G = filters.InnerOperator(wl.A, wl.B, wl.c, wl.r, wl.p)
    t_fact = time.time() - t0
    X = W_start_block(wl)
    reps = 2
    t1 = time.time()
    for _ in range(reps):
        G(X)
    t_apply = (time.time() - t1) / reps
    t_col = t_apply / X.shape[1]
    # the oracle's own count of G columns for the full solve (its per-column GMRES
    # needs many more than the block GMRES), when its full run is on file
    src = "the GPU step's count"
    golden = os.path.join(HERE, "tests", "golden", "convdiff128_eigs.txt")
    if os.path.exists(golden):
        for line in open(golden):
            if "inner_applications=" in line:
                cols_per_step = sum(json.loads(line.split("inner_applications=")[1].strip()))
                src = "the oracle's own full run, tests/golden/convdiff128_eigs.txt"
    est = t_fact + cols_per_step * t_col
    model, ncpu = host_cpu()
    # all cores: the p poles' factorizations and solves in p worker processes (the
    # oracle's band LU and solves are single-threaded C), timed end to end
    nproc = max(1, min(wl.p, ncpu))
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc) as pool:
        pool.map(_oracle_pole_term, [("w", [0], 1, 1)] * nproc)          # start the workers
        t2 = time.time()
        pool.map(_oracle_pole_term, [("w", [i], wl.seed, X.shape[1]) for i in range(wl.p)])
        t_par = time.time() - t2
    # per pole: one factorization + one application to the whole block
    t_col_par = max(t_par - t_fact / wl.p * np.ceil(wl.p / nproc), 1e-9) / X.shape[1]
    est_par = t_fact / wl.p * np.ceil(wl.p / nproc) + cols_per_step * t_col_par
    return {
        "value": float(wl.s_expected / est), "unit": "eigenpairs/s", "cores": 1,
        "kind": "oracle", "cpu": model, "cpus_available": ncpu,
        "sample": (f"oracle band LU of the {wl.p} shifted pencils ({t_fact:.1f} s) and {reps} "
                   f"applications of G to the {X.shape[1]}-column start block ({t_apply:.1f} s each), "
                   f"one thread; scaled to {wl.p} factorizations + {cols_per_step:.0f} G columns "
                   f"per solve ({src}) = {est:.0f} s for {wl.s_expected} pairs; "
                   f"orthogonalisation, least squares and projection not included"),
        "all_cores": {"value": float(wl.s_expected / est_par), "unit": "eigenpairs/s",
                      "cores": nproc,
                      "sample": (f"the same sample with the {wl.p} poles in {nproc} processes "
                                 f"({t_par:.1f} s for factorization + one application), scaled the "
                                 f"same way = {est_par:.0f} s; the oracle parallelizes over poles only")},
    }


def toeplitz_form(balanced, reps):
    """The tridiagonal Toeplitz pencil (n = 2000, a = 0, b = 1, c = 0.5 e^{i pi/3}, B = I),
    disk c = 0.3 + 0.2i enclosing 20 eigenvalues, p = q = 4, w = 32.  The balanced
    variant (normal) is checked against the closed-form eigenvalues; the literal one is
    exponentially non-normal (kappa(X) ~ 2^1000), so its pairs are pseudo-eigenpairs
    that can meet the residual bar while missing the closed form: reported as measured."""
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    wl = W.toeplitz_workload(n=2000, balanced=balanced, w=32, count=20)
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    P = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=32, expected_count=20)
    Y0 = torch.from_numpy(W.start_block(wl.n, 32, 0)).cuda()

    def step():
        P.factor_shifts()
        return P.solve_region(Y0, allow_noconv=True)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    good = (np.abs(res["lam"] - wl.c) < wl.r) & (res["err"] <= 1e-10)
    matched = 0
    if len(res["lam"]):
        d = np.abs(res["lam"][:, None] - inside[None, :]).min(axis=1)
        matched = int(np.sum(good & (d <= 1e-10 * np.abs(res["lam"]))))
    P.close()
    return {"workload": f"toeplitz_n2000_{'balanced' if balanced else 'literal'}_p4_q4_w32",
            "ms_per_step": round(ms, 3), "converged_count": int(good.sum()),
            "closed_form_matched": matched, "closed_form_inside": int(len(inside)),
            "sweeps": res["sweeps"], "krylov_steps": res["krylov_steps"],
            "value": round(int(good.sum()) / (ms / 1000.0), 3), "unit": "eigenpairs/s"}


def convdiff256_form(reps):
    """The 256 x 256 random-velocity workload (N = 65536, bandwidth 256, 187 eigenvalues
    in the disk, p = q = 8, w = 256): plain complex128 against the precision form
    (complex64 band solves, complex128 outer solves, residual form from the second
    sweep), same start block; band-solve rates of both."""
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    wl = W.convdiff256_workload()
    Y0 = torch.from_numpy(W.start_block(wl.n, wl.w, wl.seed)).cuda()
    fl_col = solve_flops_per_column(wl.n, 256, 256, wl.p)
    out = {"workload": "convdiff256_randv_p8_q8_w256", "n": wl.n, "bandwidth": 256,
           "expected_count": wl.s_expected}
    for key, prec in (("plain_c128", 0), ("precision_c64", 1)):
        P = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w,
                       expected_count=wl.s_expected, max_krylov_blocks=60, precision=prec)

        def step():
            P.factor_shifts()
            return P.solve_region(Y0, allow_noconv=True)

        step()
        torch.cuda.synchronize()
        P.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            res = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        st = P.profile_read()
        P.profile_enable(False)
        good = (np.abs(res["lam"] - wl.c) < wl.r) & (res["err"] <= 1e-10)
        t = fl_col * st["solve_columns"] / (st["solve_ms"] * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if prec == 0 else PEAK_FP32_TFLOPS
        out[key] = {"ms_per_step": round(ms, 3), "converged_count": int(good.sum()),
                    "value": round(int(good.sum()) / (ms / 1000.0), 3), "unit": "eigenpairs/s",
                    "sweeps": res["sweeps"], "krylov_steps": res["krylov_steps"],
                    "max_err": float(res["err"].max()) if len(res["err"]) else None,
                    "factor_ms": round(st["factor_ms"] / reps, 3),
                    "band_solve": {"avg_launch_ms": round(st["solve_ms"] / max(st["solve_launches"], 1), 4),
                                   "avg_columns_per_launch": round(st["solve_columns"] / max(st["solve_launches"], 1), 2),
                                   "achieved": round(t, 3), "peak": peak, "unit": "TFLOP/s",
                                   "frac": round(t / peak, 4)}}
        P.close()
    out["precision_speedup"] = round(out["plain_c128"]["ms_per_step"] / out["precision_c64"]["ms_per_step"], 3)
    return out


def batched_form(ndisks, reps):
    """Many adjacent disks of one pencil (128 x 128 constant-velocity convection-
    diffusion, B = I, closed-form spectrum): all disks' poles factorized in one
    launch sequence and the disks solved concurrently, against the same disks run
    one after another with a plan each.  Counts are checked against the closed form."""
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    A, B, disks, exact = W.disk_batch(n=128, ndisks=ndisks)
    _, kappa = W.convdiff_const_cond(128)
    specs = [{"c": d["c"], "r": d["r"], "w": d["w"], "expected_count": d["count"]}
             for d in disks]
    common = dict(p=4, q=8, max_krylov_blocks=60)
    Y0 = [torch.from_numpy(W.start_block(A.shape[0], s["w"], 100 + d)).cuda()
          for d, s in enumerate(specs)]

    def good(res, s):
        # converged pairs whose eigenvalue is the closed-form one within the
        # first-order bound kappa * residual norm (the pencil is non-normal)
        inside = np.abs(exact - s["c"]) < s["r"]
        ok = res["err"] <= 1e-10
        lam, e = res["lam"][ok], res["err"][ok]
        if len(lam) == 0:
            return 0
        j = np.abs(lam[:, None] - exact[inside][None, :]).argmin(axis=1)
        bound = 4.0 * kappa[inside][j] * e * (abs(s["c"]) + s["r"]) + 1e-13 * np.abs(lam)
        return int(np.sum(np.abs(lam - exact[inside][j]) <= bound))

    batch = rfeig.Batch(A, B, specs, **common)

    def step_batched():
        batch.factor()
        return batch.solve(Y0, allow_noconv=True)

    step_batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        outs = step_batched()
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1000.0 / reps
    found_b = sum(good(r, s) for r, s in zip(outs, specs))
    mem_b = batch.device_bytes
    batch.close()
    del batch

    plans = [rfeig.Plan(A, B, s["c"], s["r"], w=s["w"], expected_count=s["expected_count"],
                        **common) for s in specs]

    def step_seq():
        res = []
        for P, y in zip(plans, Y0):
            P.factor_shifts()
            res.append(P.solve_region(y, allow_noconv=True))
        return res

    step_seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs_s = step_seq()                 # one timed pass: a reference line, not the metric
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1000.0
    found_s = sum(good(r, s) for r, s in zip(outs_s, specs))
    for P in plans:
        P.close()
    expected = sum(s["expected_count"] for s in specs)
    return {"workload": f"convdiff128_I_{ndisks}disks_p4_q8", "disks": ndisks,
            "widths": [s["w"] for s in specs], "expected_count": expected,
            "ms_per_step": round(ms_b, 3), "value": round(found_b / (ms_b / 1000.0), 3),
            "unit": "eigenpairs/s", "converged_count": found_b,
            "sweeps": [r["sweeps"] for r in outs], "device_gb": round(mem_b / 1e9, 2),
            "sequential": {"ms_per_step": round(ms_s, 3), "converged_count": found_s,
                           "value": round(found_s / (ms_s / 1000.0), 3)}}


def batched_window_256(slots, capacity=64, trsm_cols=8):
    """The batched configuration (as batched_form_256) with a sliding window instead of
    waves: `slots` host threads, each with its own stream, take the next disk (widest
    first) as soon as their previous one is done and the window has room for it, one
    plan per disk (its own band factorization, then Alg. composite), so no disk waits for
    the slowest of a wave.  A disk of block width w takes max(w, 64) / 32 of `capacity`
    units: eight disks of width 256 at a time (223 GB), up to `slots` narrow ones.  Eight
    threads: with sixteen and four columns per solve workgroup, the HIP runtime ran out of
    resources for the scratch memory of that tile-256 solve kernel on that many streams
    (the process aborted); the eight-column kernel uses no scratch, and twelve threads ran
    but were not faster (more caching-allocator retries, 239 GB).  The band solves
    take `trsm_cols` right-hand sides per workgroup, eight by default: the plans in flight
    share the compute units, so the fewest workgroups per column win, where a lone plan's
    automatic choice (one plan after another below) takes the narrowest slices that still
    run at once, the shortest launch."""
    import queue
    import threading
    import torch
    from scipy.optimize import linear_sum_assignment
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    gdir = os.path.join(HERE, "tests", "golden")
    disks = W.read_disk_table(os.path.join(gdir, "convdiff256_disks.txt"))
    ref = np.loadtxt(os.path.join(gdir, "convdiff256_disk_eigs.txt"))
    wl = W.convdiff256_workload()
    A, B = wl.A, wl.B
    common = dict(p=4, max_krylov_blocks=40, trsm_cols=trsm_cols)

    def good(res, d):
        lam_ref = ref[ref[:, 0] == d][:, 1] + 1j * ref[ref[:, 0] == d][:, 2]
        ok = res["err"] <= 1e-10
        lam = res["lam"][ok]
        if len(lam) == 0 or len(lam_ref) == 0:
            return 0
        cost = np.abs(lam[:, None] - lam_ref[None, :])
        r_, c_ = linear_sum_assignment(cost)
        return int(np.sum(cost[r_, c_] <= 1e-10 * np.abs(lam_ref[c_])))

    todo = queue.Queue()
    for d in sorted(range(len(disks)), key=lambda d: (-disks[d]["w"], d)):
        todo.put(d)
    found, sweeps, errors = {}, {}, []
    lock = threading.Lock()
    room = threading.Condition(lock)
    live = [0, 0, 0]                               # bytes of the plans alive, peak, units in use

    def worker():
        st = torch.cuda.Stream()
        while True:
            try:
                d = todo.get_nowait()
            except queue.Empty:
                return
            dk = disks[d]
            units = max(dk["w"], 64) // 32
            with room:
                while live[2] + units > capacity:
                    room.wait()
                live[2] += units
            try:
                with torch.cuda.stream(st):
                    P = rfeig.Plan(A, B, dk["c"], dk["r"], w=dk["w"], q=dk["q"],
                                   expected_count=dk["count"], stream=st, **common)
                    nb = P.device_bytes
                    with lock:
                        live[0] += nb
                        live[1] = max(live[1], live[0])
                    P.factor_shifts()
                    y = torch.from_numpy(W.start_block(wl.n, dk["w"], 100 + d)).cuda()
                    r = P.solve_region(y, allow_noconv=True)
                    found[d] = good(r, d)
                    sweeps[d] = r["sweeps"]
                    P.close()
                    with lock:
                        live[0] -= nb
            except Exception as e:                 # reported in the result
                errors.append((d, repr(e)))
            with room:
                live[2] -= units
                room.notify_all()

    torch.cuda.synchronize()
    retries0 = torch.cuda.memory_stats().get("num_alloc_retries", 0)
    t0 = time.perf_counter()
    threads = [threading.Thread(target=worker) for _ in range(slots)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0
    total = int(sum(found.values()))
    out = {"workload": f"convdiff256_randv_{len(disks)}disks_p4_q4-8-16", "disks": len(disks),
           "slots": slots, "capacity_units": capacity,
           "expected_count": int(sum(d["count"] for d in disks)),
           "ms_per_step": round(ms, 3), "value": round(total / (ms / 1000.0), 3),
           "unit": "eigenpairs/s", "converged_count": total,
           "sweeps": [sweeps.get(d) for d in range(len(disks))],
           "peak_device_gb": round(live[1] / 1e9, 2),
           "alloc_retries": int(torch.cuda.memory_stats().get("num_alloc_retries", 0) - retries0)}
    if errors:
        out["errors"] = errors[:4]
    return out


def batched_form_256(wave, with_sequential=True, mode="window"):
    """The batched configuration: 64 disks along the real axis of the 256 x 256
    random-velocity pencil (10..200 eigenvalues each, block widths 16..256, p = 4,
    q cycling through 4, 8, 16; tests/golden/convdiff256_disks.txt).  mode "window": a
    sliding window of `wave` disks in flight (batched_window_256); mode "wave": the
    disks go through the HBM in waves of `wave` disks of similar block width, per wave
    one batch (all its poles factorized in one launch sequence, its disks solved
    concurrently on their own streams), destroyed before the next.  A pair counts when it is converged
    (inside, e <= 1e-10) and matches the oracle's reference eigenvalue of its disk
    to 1e-10 relative (tests/golden/convdiff256_disk_eigs.txt).  Against the same
    disks solved one after another, one plan each."""
    import torch
    from scipy.optimize import linear_sum_assignment
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    gdir = os.path.join(HERE, "tests", "golden")
    disks = W.read_disk_table(os.path.join(gdir, "convdiff256_disks.txt"))
    ref = np.loadtxt(os.path.join(gdir, "convdiff256_disk_eigs.txt"))
    wl = W.convdiff256_workload()
    A, B = wl.A, wl.B
    common = dict(p=4, max_krylov_blocks=40)

    def good(res, d):
        lam_ref = ref[ref[:, 0] == d][:, 1] + 1j * ref[ref[:, 0] == d][:, 2]
        ok = res["err"] <= 1e-10
        lam = res["lam"][ok]
        if len(lam) == 0 or len(lam_ref) == 0:
            return 0
        cost = np.abs(lam[:, None] - lam_ref[None, :])
        r_, c_ = linear_sum_assignment(cost)
        return int(np.sum(cost[r_, c_] <= 1e-10 * np.abs(lam_ref[c_])))

    def y0(d):
        return torch.from_numpy(W.start_block(wl.n, disks[d]["w"], 100 + d)).cuda()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    found_b, sweeps, peak = 0, [], 0
    # waves of disks of similar block width (a wave lasts as long as its slowest disk)
    order = sorted(range(len(disks)), key=lambda d: (-disks[d]["w"], d))
    for w0 in (range(0, len(disks), wave) if mode == "wave" else []):
        idx = order[w0:w0 + wave]
        specs = [{"c": disks[d]["c"], "r": disks[d]["r"], "w": disks[d]["w"], "q": disks[d]["q"],
                  "expected_count": disks[d]["count"]} for d in idx]
        bt = rfeig.Batch(A, B, specs, **common)
        peak = max(peak, bt.device_bytes)
        bt.factor()
        outs = bt.solve([y0(d) for d in idx], allow_noconv=True)
        for d, r in zip(idx, outs):
            found_b += good(r, d)
            sweeps.append(r["sweeps"])
        bt.close()
        del bt
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1000.0
    if mode == "window":
        win = batched_window_256(wave)
        ms_b, found_b, sweeps = win["ms_per_step"], win["converged_count"], win["sweeps"]
        peak = win["peak_device_gb"] * 1e9
    expected = int(sum(d["count"] for d in disks))
    out = {"workload": f"convdiff256_randv_{len(disks)}disks_p4_q4-8-16", "disks": len(disks),
           "mode": mode, ("slots" if mode == "window" else "wave"): wave,
           "widths": [d["w"] for d in disks], "expected_count": expected,
           "ms_per_step": round(ms_b, 3), "value": round(found_b / (ms_b / 1000.0), 3),
           "unit": "eigenpairs/s", "converged_count": found_b, "sweeps": sweeps,
           "peak_batch_device_gb": round(peak / 1e9, 2)}
    if mode == "window":
        out["alloc_retries"] = win["alloc_retries"]     # caching-allocator frees and retries
    if with_sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        found_s = 0
        for d, dk in enumerate(disks):
            P = rfeig.Plan(A, B, dk["c"], dk["r"], w=dk["w"], q=dk["q"], expected_count=dk["count"],
                           **common)
            P.factor_shifts()
            found_s += good(P.solve_region(y0(d), allow_noconv=True), d)
            P.close()
        torch.cuda.synchronize()
        ms_s = (time.perf_counter() - t0) * 1000.0
        out["sequential"] = {"ms_per_step": round(ms_s, 3), "converged_count": found_s,
                             "value": round(found_s / (ms_s / 1000.0), 3)}
        out["batched_speedup"] = round(ms_s / ms_b, 3)
    return out


def circuit_form(reps):
    """The paper's circuit pencil (App. B) at n_x = 10 (N = 1220), its solver shape
    (k1 = k2 = 8, n_col = 24) and a disk with 17 eigenvalues: Alg. composite."""
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    wl = W.circuit_workload()
    P = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w, expected_count=wl.s_expected)
    Y0 = torch.from_numpy(W.start_block(wl.n, wl.w, 0)).cuda()

    def step():
        P.factor_shifts()
        return P.solve_region(Y0, allow_noconv=True)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    good = int(np.sum((np.abs(res["lam"] - wl.c) < wl.r) & (res["err"] <= 1e-10)))
    P.close()
    return {"workload": "circuit_nx10_p8_q8_w24", "n": wl.n, "expected_count": wl.s_expected,
            "converged_count": good, "sweeps": res["sweeps"], "krylov_steps": res["krylov_steps"],
            "ms_per_step": round(ms, 3), "value": round(good / (ms / 1000.0), 3),
            "unit": "eigenpairs/s"}


def gradient_form(reps):
    """Eigenvalue gradients on the 128 x 128 random-velocity pencil (52 eigenvalues in
    the disk): one band factorization, right eigenpairs (Alg. composite), left
    eigenpairs from the adjoint pencil (Alg. composite whose solves are the K_i^H sweeps
    over the same factors, transposed once), and the device contraction of
    d lambda_i / d A over the stored entries of A and B for one weight vector."""
    import torch
    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W
    wl = W.random_velocity_workload()
    opts = dict(p=wl.p, q=wl.q, w=wl.w, expected_count=wl.s_expected, max_krylov_blocks=60)
    P = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, **opts)
    Pa = P.adjoint(stream=torch.cuda.Stream())
    Y0 = torch.from_numpy(W.start_block(wl.n, wl.w, 0)).cuda()
    Y0a = torch.from_numpy(W.start_block(wl.n, wl.w, 1)).cuda()

    def step():
        # one factorization (the adjoint plan transposes its tiles), then the right and
        # adjoint problems solved concurrently on two streams
        t0 = time.perf_counter()
        res, resa = rfeig.solve_regions([P, Pa], [Y0, Y0a], factor=True, allow_noconv=True)
        t2 = time.perf_counter()
        g = np.ones(res["count"], np.complex128)
        P.eig_vjp(res["lam"], res["X"], resa["lam"], resa["X"], g, wl.A.nnz, wl.B.nnz)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return res, resa, (t2 - t0, 0.0, t3 - t2)

    step()
    tot = np.zeros(3)
    for _ in range(reps):
        res, resa, t = step()
        tot += np.array(t)
    ms = tot * 1000.0 / reps
    n_ok = int(np.sum(res["err"] <= 1e-10))
    out = {"workload": "convdiff128_randv_p4_q8_w64", "expected_count": wl.s_expected,
           "count": res["count"], "count_adjoint": resa["count"],
           "ms_right_and_adjoint": round(ms[0], 3), "ms_vjp": round(ms[2], 3),
           "ms_per_step": round(ms.sum(), 3),
           "value": round(n_ok / (ms.sum() / 1000.0), 3), "unit": "eigenvalue gradients/s"}
    P.close()
    Pa.close()
    return out


def W_start_block(wl):
    from paper_2310_18043_amd import workloads as W
    return W.start_block(wl.n, wl.w, wl.seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # five timed steps: the host QZ of the last sweep is on the step's critical path and
    # its time varies with the host's load, so a few more steps steady the average
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--subblock", type=int, default=0)
    ap.add_argument("--trsm-cols", type=int, default=0)
    ap.add_argument("--solve-form", type=int, default=0,
                    help="band solves: 0 cluster form where it applies (tiles 64, 128), 1 per slice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adaptive-qmax", type=int, default=64,
                    help="also time Alg. composite2 up to this outer node count (0: skip)")
    ap.add_argument("--batch-disks", type=int, default=64,
                    help="also time the batched form on this many disks (0: skip)")
    ap.add_argument("--no-circuit", action="store_true",
                    help="skip the circuit-pencil measurement")
    ap.add_argument("--no-c64", action="store_true",
                    help="skip the precision-form (complex64 band solves) measurement")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip the differentiation-form measurement")
    ap.add_argument("--no-convdiff256", action="store_true",
                    help="skip the 256 x 256 workload (plain and precision form)")
    ap.add_argument("--no-toeplitz", action="store_true",
                    help="skip the Toeplitz workload (balanced and literal)")
    ap.add_argument("--batch256-wave", type=int, default=8,
                    help="disks in flight (window) or per wave of the 64-disk 256 x 256 "
                         "batched workload (0: skip)")
    ap.add_argument("--batch256-mode", choices=("window", "wave"), default="window",
                    help="the batched 256 x 256 workload: a sliding window of disks in flight, "
                         "or waves of batches")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(the per-GPU shard is the whole problem); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calib_copy:
        a = torch.empty(1 << 26, dtype=torch.complex128, device="cuda")   # 1 GiB
        a.zero_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": a.numel() * 16, "copies": 3}))
        return

    from paper_2310_18043_amd import rfeig
    from paper_2310_18043_amd import workloads as W

    wl = W.convdiff_workload()
    kl, ku = 128, 128
    props = torch.cuda.get_device_properties(0)
    log(f"device {props.name} {getattr(props, 'gcnArchName', '')} CUs={props.multi_processor_count} "
        f"lds/block={getattr(props, 'shared_memory_per_block', '?')} "
        f"lds/cu={getattr(props, 'shared_memory_per_multiprocessor', '?')}")
    log(f"workload {wl.name}: n={wl.n} p={wl.p} q={wl.q} w={wl.w} disk c={wl.c} r={wl.r:.3f}")
    plan = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w,
                      expected_count=wl.s_expected, subblock=args.subblock,
                      trsm_cols=args.trsm_cols, solve_form=args.solve_form)
    Y0 = torch.from_numpy(W.start_block(wl.n, wl.w, wl.seed)).cuda()
    Y0 = rfeig.as_colmajor(Y0)
    torch.cuda.synchronize()

    def step():
        plan.factor_shifts()
        return plan.solve_region(Y0, allow_noconv=True)

    for i in range(args.warmup):
        t = time.time()
        res = step()
        log(f"warmup {i}: {time.time() - t:.3f} s, count={res['count']}, sweeps={res['sweeps']}, "
            f"krylov={res['krylov_steps']}")
    plan.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = plan.profile_read()
    plan.profile_enable(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    res = results[-1]
    good = (np.abs(res["lam"] - wl.c) < wl.r) & (res["err"] <= 1e-10)
    count = int(good.sum())
    log(f"timed: {ms_per_step:.1f} ms/step, converged pairs {count}, sweeps {res['sweeps']}, "
        f"krylov steps {res['krylov_steps']}, filter {res['ms_filter']:.1f} ms, hsrr {res['ms_hsrr']:.1f} ms")
    log(f"kernel stats: {stats}")

    # dominant kernel: band solve (G)
    fl_col = solve_flops_per_column(wl.n, kl, ku, wl.p)
    achieved_tflops = fl_col * stats["solve_columns"] / (stats["solve_ms"] * 1e-3) / 1e12
    avg_cols = stats["solve_columns"] / max(stats["solve_launches"], 1)
    # tiles 64 and 128 solve with the cluster kernel (FP64 matrix cores), others per slice
    tile = 16
    while tile < max(kl, ku):
        tile *= 2
    cluster = tile in (64, 128) and args.solve_form == 0
    kname = "band_solve_cluster_kernel" if cluster else "band_solve_kernel"
    tfile = TRAFFIC_FILES[kname]
    traffic = None
    if os.path.exists(tfile):
        try:
            traffic = json.load(open(tfile)).get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {
        "kernel": kname,
        "bound": "mfma" if cluster else "alu",
        "achieved": round(achieved_tflops, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved_tflops / PEAK_FP64_TFLOPS, 4),
        "traffic": traffic,
        "traffic_source": (f"stored: profiles/{os.path.basename(tfile)}, rocprofv3 FETCH_SIZE "
                           "and WRITE_SIZE passes of this bench command on the same kernel, scaled "
                           "by a 1 GiB copy") if traffic is not None else None,
        "avg_launch_ms": round(stats["solve_ms"] / max(stats["solve_launches"], 1), 4),
        "launches": stats["solve_launches"],
        "avg_columns_per_launch": round(avg_cols, 2),
        "algorithmic_flops_per_launch": fl_col * avg_cols,
        "algorithmic_bytes_per_launch": solve_bytes_per_launch(wl.n, kl, ku, wl.p, avg_cols),
    }

    # one composite filter application on the start block (the first sweep's input)
    Yc = Y0
    torch.cuda.synchronize()
    plan.profile_enable(True)
    tf0 = time.perf_counter()
    U, finfo = plan.filter_apply(Yc, allow_noconv=True)
    torch.cuda.synchronize()
    tf = time.perf_counter() - tf0
    fstats = plan.profile_read()
    plan.profile_enable(False)
    m = finfo["krylov_steps"]
    b = plan.opts.subblock or 32
    # work model: G on all applied columns + block Gram-Schmidt/CholQR + combine
    n, w, p, s = wl.n, wl.w, wl.p, 16
    g_flops = fl_col * finfo["inner_columns"]
    gs_flops = 16.0 * n * b * w * m * (m + 1) + 32.0 * n * b * w * m
    comb_flops = 8.0 * n * m * b * w
    f_bytes = (fstats["solve_launches"] * p * ((2 * kl + ku + 1) * n * 16 + 4 * n)
               + finfo["inner_columns"] * n * 16 * (1 + p)
               + 2.0 * n * w * s * m * (m + 1) + 8.0 * n * w * s * m + n * (m + 1) * w * s)
    fa = {
        "ms": round(tf * 1000, 3), "krylov_steps": m, "inner_columns": finfo["inner_columns"],
        "algorithmic_tflops": round((g_flops + gs_flops + comb_flops) / tf / 1e12, 3),
        "frac_fp64_peak": round((g_flops + gs_flops + comb_flops) / tf / 1e12 / PEAK_FP64_TFLOPS, 4),
        "algorithmic_gbps": round(f_bytes / tf / 1e9, 1),
        "frac_hbm_peak": round(f_bytes / tf / 1e9 / PEAK_HBM_GBPS, 4),
        "max_residual": finfo["max_residual"],
    }
    log(f"filter_apply: {fa}")

    # Alg. composite2 on the same workload and start block: outer node count doubling
    # from q to q_max on one Krylov basis, no subspace iteration
    c2 = None
    if args.adaptive_qmax > 0:
        plan2 = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w,
                           expected_count=wl.s_expected, q_max=args.adaptive_qmax,
                           max_krylov_blocks=60, subblock=args.subblock)

        def step2():
            plan2.factor_shifts()
            return plan2.solve_region_adaptive(Y0, allow_noconv=True)

        step2()
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        reps2 = max(1, min(args.steps, 2))
        for _ in range(reps2):
            r2 = step2()
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - tc0) * 1000.0 / reps2
        good2 = (np.abs(r2["lam"] - wl.c) < wl.r) & (r2["err"] <= 1e-10)
        c2 = {"ms_per_step": round(ms2, 3),
              "value": round(int(good2.sum()) / (ms2 / 1000.0), 3), "unit": "eigenpairs/s",
              "converged_count": int(good2.sum()), "levels": r2["sweeps"],
              "q_levels": [wl.q * 2 ** i for i in range(r2["sweeps"])],
              "basis_depth": r2["krylov_steps"], "q_max": args.adaptive_qmax,
              "ms_filter": round(r2["ms_filter"], 3), "ms_hsrr": round(r2["ms_hsrr"], 3)}
        log(f"composite2: {c2}")
        del plan2

    # precision form on the same workload and start block: complex64 band solves,
    # complex128 outer solves, projections and residuals
    pc = None
    if not args.no_c64:
        plan3 = rfeig.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w,
                           expected_count=wl.s_expected, subblock=args.subblock, precision=1)

        def step3():
            plan3.factor_shifts()
            return plan3.solve_region(Y0, allow_noconv=True)

        step3()
        torch.cuda.synchronize()
        plan3.profile_enable(True)
        tc0 = time.perf_counter()
        reps3 = max(1, min(args.steps, 2))
        for _ in range(reps3):
            r3 = step3()
        torch.cuda.synchronize()
        ms3 = (time.perf_counter() - tc0) * 1000.0 / reps3
        st3 = plan3.profile_read()
        plan3.profile_enable(False)
        good3 = (np.abs(r3["lam"] - wl.c) < wl.r) & (r3["err"] <= 1e-10)
        cols3 = st3["solve_columns"] / max(st3["solve_launches"], 1)
        t3 = fl_col * st3["solve_columns"] / (st3["solve_ms"] * 1e-3) / 1e12
        pc = {"ms_per_step": round(ms3, 3), "value": round(int(good3.sum()) / (ms3 / 1000.0), 3),
              "unit": "eigenpairs/s", "converged_count": int(good3.sum()), "sweeps": r3["sweeps"],
              "krylov_steps": r3["krylov_steps"], "ms_filter": round(r3["ms_filter"], 3),
              "ms_hsrr": round(r3["ms_hsrr"], 3),
              "factor_ms": round(st3["factor_ms"] / reps3, 3),
              "band_solve_c64": {"avg_launch_ms": round(st3["solve_ms"] / max(st3["solve_launches"], 1), 4),
                                 "avg_columns_per_launch": round(cols3, 2),
                                 "achieved": round(t3, 3), "peak": PEAK_FP32_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(t3 / PEAK_FP32_TFLOPS, 4)}}
        log(f"precision form (c64 solves): {pc}")
        del plan3

    bt = None
    if args.batch_disks > 0:
        bt = batched_form(args.batch_disks, min(args.steps, 2))
        log(f"batched: {bt}")

    circ = None
    if not args.no_circuit:
        circ = circuit_form(min(args.steps, 2))
        log(f"circuit: {circ}")

    grad = None
    if not args.no_gradient:
        grad = gradient_form(min(args.steps, 2))
        log(f"gradient: {grad}")

    bt256 = None
    if args.batch256_wave > 0 and os.path.exists(os.path.join(HERE, "tests", "golden",
                                                              "convdiff256_disks.txt")):
        bt256 = batched_form_256(args.batch256_wave, mode=args.batch256_mode)
        log(f"batched 256: { {k: v for k, v in bt256.items() if k not in ('widths', 'sweeps')} }")

    cd256 = None
    if not args.no_convdiff256:
        cd256 = convdiff256_form(min(args.steps, 2))
        log(f"convdiff256: {cd256}")

    toep = None
    if not args.no_toeplitz:
        toep = [toeplitz_form(True, min(args.steps, 2)), toeplitz_form(False, min(args.steps, 2))]
        log(f"toeplitz: {toep}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(wl, stats["solve_columns"] / max(args.steps, 1))
        log(f"cpu baseline: {cpu}")

    value = count / (ms_per_step / 1000.0)
    line = {
        "metric": "converged eigenpairs/s at residual \u22641e-10; filter_apply GB/s & % FP64 peak",
        "value": round(value, 3),
        "unit": "eigenpairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": "convdiff128_upwind_p4_q8_w128", "n": wl.n, "bandwidth": kl,
                   "p": wl.p, "q": wl.q, "w": wl.w, "disk_c": [wl.c.real, wl.c.imag],
                   "disk_r": wl.r, "expected_count": wl.s_expected,
                   "converged_count": count, "sweeps": res["sweeps"],
                   "krylov_steps": res["krylov_steps"],
                   "subblock": b, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "filter_apply": fa,
        "composite2": c2,
        "precision_c64": pc,
        "batched": bt,
        "gradient": grad,
        "circuit": circ,
        "convdiff256": cd256,
        "batched_256": bt256,
        "toeplitz": toep,
        "phases_ms": {"factor": round(stats["factor_ms"] / max(args.steps, 1), 3),
                      "filter": round(res["ms_filter"], 3), "hsrr": round(res["ms_hsrr"], 3)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
