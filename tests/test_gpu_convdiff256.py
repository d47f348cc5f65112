"""GPU parity on the 256 x 256 random-velocity workload (N = 65536, bandwidth 256,
per-cell velocity U[-30, 30]^2, 187 eigenvalues in the disk, p = q = 8, w = 256), in
the launch shapes the benchmark times: plain complex128 and the precision form.

References (tests/golden/make_convdiff256.py, oracle only): the eigenvalues inside the
disk (shift-invert Arnoldi refined by two-sided inverse iteration) with their
condition numbers kappa_B (1.0 .. 20), and 128-vector Gaussian sketches plus exact
column norms of G(X) (simple rule with p poles) and of the filter (simple rule with pq
poles) on the 256-column blocks.

Bars: G per column 1e-12; filter per column max(1e-12, 16 max(kappa_B) u) (as on the
128 x 128 workload); eigenvalues 1e-10 relative over a minimum-cost assignment and
within the first-order bound kappa_B (residual norm) + 1e-12 |lambda|; residuals
<= 1e-10 re-evaluated by the oracle's definition.  The precision form must meet the
same eigenpair bars; its per-pair error against the oracle is printed.
"""
import os
import sys

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U_ROUND = np.finfo(np.float64).eps / 2


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def rf(torch_cuda):
    from paper_2310_18043_amd import rfeig
    return rfeig


@pytest.fixture(scope="module")
def golden():
    rows = np.loadtxt(os.path.join(HERE, "convdiff256_eigs.txt"))
    g = np.load(os.path.join(HERE, "convdiff256_sketch.npz"))
    return rows[:, 0] + 1j * rows[:, 1], rows[:, 2], g


@pytest.fixture(scope="module")
def wl():
    return W.convdiff256_workload()


def _sketch_err(U, sketch, seed):
    S = W.start_block(U.shape[0], 128, seed)
    sk = S.conj().T @ U
    return np.linalg.norm(sk - sketch, axis=0) / np.linalg.norm(sketch, axis=0)


def _plan(rf, wl, **kw):
    return rf.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w, expected_count=wl.s_expected,
                   max_krylov_blocks=60, **kw)


def test_g_and_filter_all_columns(rf, torch_cuda, wl, golden):
    lam_ref, kap, g = golden
    plan = _plan(rf, wl, gmres_tol=1e-13)
    plan.factor_shifts()
    _say("convdiff256 G, 256 columns")
    X = W.start_block(wl.n, wl.w, int(g["g_seed"]))
    Z = plan.apply_inner(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
    e = _sketch_err(Z, g["g_sketch"], int(g["sketch_seed"]))
    nz = np.abs(np.linalg.norm(Z, axis=0) / g["g_norms"] - 1).max()
    print(f"convdiff256 G: per-column sketched error max {e.max():.2e} median {np.median(e):.2e}, "
          f"norm deviation {nz:.1e}")
    assert e.max() <= 1e-12 and nz <= 1e-12
    _say("convdiff256 filter_apply, 256 columns")
    Y = W.start_block(wl.n, wl.w, int(g["f_seed"]))
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    assert info["converged"]
    Uh = U.cpu().numpy()
    e = _sketch_err(Uh, g["f_sketch"], int(g["sketch_seed"]))
    nu = np.abs(np.linalg.norm(Uh, axis=0) / g["f_norms"] - 1).max()
    bar = max(1e-12, 16.0 * kap.max() * U_ROUND)
    print(f"convdiff256 filter: per-column sketched error max {e.max():.2e} median {np.median(e):.2e}, "
          f"norm deviation {nu:.1e}, krylov steps {info['krylov_steps']}; bar {bar:.1e}")
    assert e.max() <= bar and nu <= bar
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_region_vs_reference(rf, torch_cuda, wl, golden, precision):
    from oracle import hsrr
    from scipy.optimize import linear_sum_assignment
    lam_ref, kap, _ = golden
    plan = _plan(rf, wl, precision=precision)
    _say(f"convdiff256 solve_region precision={precision}")
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(wl.n, wl.w, wl.seed)).cuda())
    assert res["converged"] and res["count"] == len(lam_ref) == wl.s_expected
    lam = res["lam"]
    cost = np.abs(lam[:, None] - lam_ref[None, :])
    r_, c_ = linear_sum_assignment(cost)
    rel = cost[r_, c_] / np.abs(lam_ref[c_])
    # residual norms ||A x - lambda B x|| of the unit vectors, by the oracle's definition
    Xh = res["X"].cpu().numpy()
    e = hsrr.rel_errors(wl.A, wl.B, lam, Xh, wl.c, wl.r)
    rn = e * (abs(wl.c) + wl.r) * np.linalg.norm(wl.B @ Xh, axis=0)
    bound = kap[c_] * rn[r_] + 1e-12 * np.abs(lam_ref[c_])
    print(f"convdiff256 precision={precision}: sweeps {res['sweeps']}, max |dlambda|/|lambda| "
          f"{rel.max():.2e} (median {np.median(rel):.2e}), max residual {e.max():.2e}, "
          f"max ratio to the kappa_B bound {(cost[r_, c_] / bound).max():.2f}")
    assert rel.max() <= 1e-10, rel.max()
    assert e.max() <= 1e-10, e.max()
    assert np.all(cost[r_, c_] <= bound)
    plan.close()
