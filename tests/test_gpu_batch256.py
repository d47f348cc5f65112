"""The batched form on its stated workload: 64 disks along the real axis of the
256 x 256 random-velocity pencil (10..200 eigenvalues each, block widths 16..256,
p = 4, q cycling through 4, 8, 16), in waves of 8 disks per batch so that factors
and Krylov bases fit the HBM.  References: tests/golden/make_convdiff256_batch.py
(oracle only): each disk's eigenvalues (shift-invert Arnoldi refined by two-sided
inverse iteration) with kappa_B.

Bars per disk: the converged count equals the reference count; eigenvalues within
1e-10 relative of the references (minimum-cost assignment) and within
kappa_B * residual norm + 1e-12 |lambda|; residuals <= 1e-10 re-evaluated by the
oracle's definition.  Two disks are also solved by stand-alone plans: the batch must
give the same eigenvalues to 1e-12 relative.
"""
import os
import sys

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
WAVE = 8


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


def _refs():
    disks = W.read_disk_table(os.path.join(GOLDEN, "convdiff256_disks.txt"))
    ref = np.loadtxt(os.path.join(GOLDEN, "convdiff256_disk_eigs.txt"))
    return disks, ref


def test_64_disks_in_waves_match_references(rf, torch_cuda):
    from oracle import hsrr
    from scipy.optimize import linear_sum_assignment
    disks, ref = _refs()
    assert len(disks) == 64
    wl = W.convdiff256_workload()
    worst_rel, worst_res, total = 0.0, 0.0, 0
    for w0 in range(0, len(disks), WAVE):
        idx = list(range(w0, min(w0 + WAVE, len(disks))))
        specs = [{"c": disks[d]["c"], "r": disks[d]["r"], "w": disks[d]["w"], "q": disks[d]["q"],
                  "expected_count": disks[d]["count"]} for d in idx]
        _say(f"batch of disks {idx[0]}..{idx[-1]} (widths {[s['w'] for s in specs]})")
        bt = rf.Batch(wl.A, wl.B, specs, p=4, max_krylov_blocks=40)
        bt.factor()
        Y0 = [torch_cuda.from_numpy(W.start_block(wl.n, disks[d]["w"], 100 + d)).cuda() for d in idx]
        outs = bt.solve(Y0)
        for d, res in zip(idx, outs):
            sel = ref[:, 0] == d
            lam_ref, kap = ref[sel, 1] + 1j * ref[sel, 2], ref[sel, 3]
            assert res["converged"] and res["count"] == len(lam_ref) == disks[d]["count"], d
            lam = res["lam"]
            cost = np.abs(lam[:, None] - lam_ref[None, :])
            r_, c_ = linear_sum_assignment(cost)
            rel = cost[r_, c_] / np.abs(lam_ref[c_])
            Xh = res["X"].cpu().numpy()
            e = hsrr.rel_errors(wl.A, wl.B, lam, Xh, disks[d]["c"], disks[d]["r"])
            rn = e * (abs(disks[d]["c"]) + disks[d]["r"]) * np.linalg.norm(wl.B @ Xh, axis=0)
            assert rel.max() <= 1e-10, (d, rel.max())
            assert e.max() <= 1e-10, (d, e.max())
            assert np.all(cost[r_, c_] <= kap[c_] * rn[r_] + 1e-12 * np.abs(lam_ref[c_])), d
            worst_rel, worst_res = max(worst_rel, rel.max()), max(worst_res, e.max())
            total += res["count"]
        bt.close()
    print(f"64 disks: {total} eigenpairs, max |dlambda|/|lambda| {worst_rel:.2e}, "
          f"max residual {worst_res:.2e}")


def test_batch_disks_equal_stand_alone_plans(rf, torch_cuda):
    disks, _ = _refs()
    wl = W.convdiff256_workload()
    idx = [0, 5]                       # a small and a wider disk, different q
    specs = [{"c": disks[d]["c"], "r": disks[d]["r"], "w": disks[d]["w"], "q": disks[d]["q"],
              "expected_count": disks[d]["count"]} for d in idx]
    _say("batch of 2 disks vs stand-alone plans")
    bt = rf.Batch(wl.A, wl.B, specs, p=4, max_krylov_blocks=40)
    bt.factor()
    Y0 = [torch_cuda.from_numpy(W.start_block(wl.n, disks[d]["w"], 100 + d)).cuda() for d in idx]
    outs = bt.solve(Y0)
    bt.close()
    for d, y, ob in zip(idx, Y0, outs):
        P = rf.Plan(wl.A, wl.B, disks[d]["c"], disks[d]["r"], p=4, q=disks[d]["q"], w=disks[d]["w"],
                    expected_count=disks[d]["count"], max_krylov_blocks=40, tuned=False)
        res = P.solve_region(y)
        P.close()
        assert res["count"] == ob["count"]
        a, b = np.sort_complex(res["lam"]), np.sort_complex(ob["lam"])
        assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b)), (d, np.abs(a - b).max())
