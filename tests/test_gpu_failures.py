"""Failure handling of the C ABI on the GPU (the failure modes of Sec. 3.2 and Sec. 6:
outer solves that stop at their cap, bad input, eigenvalues on the contour, a block
too narrow for the eigenvalue count).  Every condition is forced from the host; no
kernel is made to fault.  The singular pole (RF_ERR_SINGULAR) and the sweep cap are
covered in test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _colerr(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def test_gmres_cap_reports_noconv_with_the_capped_filter(rf, torch_cuda):
    # two block-Arnoldi steps cannot reach 1e-13 on this pencil: RF_ERR_NOCONV, and the
    # block still holds the capped iterate (finite, converged flag cleared)
    from oracle import filters
    A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=1)
    c, r = 900 + 0.05j, 250.0
    _say("filter_apply with max_krylov_blocks = 2")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=16, gmres_tol=1e-13, max_krylov_blocks=2)
    plan.factor_shifts()
    Y = torch_cuda.from_numpy(W.start_block(A.shape[0], 16, seed=3)).cuda()
    with pytest.raises(rf.RfError) as ei:
        plan.filter_apply(Y)
    assert ei.value.status == rf.RF_ERR_NOCONV
    U, info = plan.filter_apply(Y, allow_noconv=True)
    assert not info["converged"] and info["krylov_steps"] == 2
    assert info["max_residual"] > 1e-13
    Uh = U.cpu().numpy()
    assert np.all(np.isfinite(Uh))
    # a plan with room for the outer solves converges on the same block
    ok = rf.Plan(A, B, c, r, p=4, q=8, w=16, gmres_tol=1e-13)
    ok.factor_shifts()
    U2, info2 = ok.filter_apply(Y)
    assert info2["converged"]
    ref = filters.simple_filter(A, B, c, r, 32, Y.cpu().numpy())
    assert _colerr(U2.cpu().numpy(), ref).max() < _colerr(Uh, ref).max()


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_block_is_rejected_and_the_plan_stays_usable(rf, torch_cuda, bad):
    from oracle import filters
    A, B = W.convdiff_pencil(16, mass=(0.5, 1.5), seed=2)
    c, r = 700 + 0.05j, 200.0
    _say(f"filter_apply / solve_region with {bad} in the block")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=8, gmres_tol=1e-13)
    plan.factor_shifts()
    Yh = W.start_block(A.shape[0], 8, seed=4)
    Ybad = Yh.copy()
    Ybad[17, 5] = bad
    with pytest.raises(rf.RfError) as ei:
        plan.filter_apply(torch_cuda.from_numpy(Ybad).cuda())
    assert ei.value.status == rf.RF_ERR_ARG and "column 5" in str(ei.value)
    with pytest.raises(rf.RfError) as ei:
        plan.solve_region(torch_cuda.from_numpy(Ybad).cuda())
    assert ei.value.status == rf.RF_ERR_ARG
    # nothing was left half done: the same plan still filters a good block correctly
    U, info = plan.filter_apply(torch_cuda.from_numpy(Yh).cuda())
    ref = filters.simple_filter(A, B, c, r, 32, Yh)
    assert info["converged"] and _colerr(U.cpu().numpy(), ref).max() <= 1e-12


def test_eigenvalues_within_1e12_of_the_contour(rf, torch_cuda):
    # diagonal pencil (normal) with eigenvalues at relative distance 1e-12 inside and
    # outside the circle: the filter value there is 1/2, so both stay in the filtered
    # subspace; every pair the solver returns is exact to its residual, every eigenvalue
    # well inside is found, and the two on the rim are classified by the strict test
    # |lambda - c| < r of their computed value (they may fall either way).
    rng = np.random.default_rng(11)
    c, r = 0.5 + 0.25j, 1.0
    inner = c + 0.8 * r * np.sqrt(rng.uniform(0, 1, 10)) * np.exp(2j * np.pi * rng.uniform(0, 1, 10))
    rim = c + r * np.array([1 - 1e-12, 1 + 1e-12]) * np.exp(1j * np.array([0.3, 2.1]))
    outer = c + r * rng.uniform(1.3, 4.0, 300) * np.exp(2j * np.pi * rng.uniform(0, 1, 300))
    lam = np.concatenate([inner, rim, outer])
    bd = rng.uniform(0.5, 1.5, lam.size)
    A, B = W.diagonal_pencil(lam, bd)
    _say("solve_region with eigenvalues 1e-12 from the contour")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=24)
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(lam.size, 24, 0)).cuda(),
                            allow_noconv=True)
    got = res["lam"]
    d = np.abs(got[:, None] - lam[None, :]).min(axis=1)
    assert np.all(d <= 1e-9), d.max()
    assert np.all(np.abs(got - c) < r)
    for z in inner:
        assert np.abs(got - z).min() <= 1e-9 * abs(z)
    print("rim pairs returned:", int(sum(np.abs(got - z).min() <= 1e-9 for z in rim)),
          "status converged:", res["converged"], "sweeps", res["sweeps"])


def test_block_narrower_than_the_count(rf, torch_cuda):
    # 20 eigenvalues inside D but only w = 8 columns: the subspace cannot hold them, so
    # the stopping rule is never met (RF_ERR_NOCONV after the sweep cap) or the pairs
    # it returns are still exact eigenpairs; never a wrong pair.
    rng = np.random.default_rng(12)
    c, r = 0.0, 1.0
    inside = 0.9 * np.sqrt(rng.uniform(0, 1, 20)) * np.exp(2j * np.pi * rng.uniform(0, 1, 20))
    outside = rng.uniform(1.3, 4.0, 200) * np.exp(2j * np.pi * rng.uniform(0, 1, 200))
    lam = np.concatenate([inside, outside])
    A, B = W.diagonal_pencil(lam)
    _say("solve_region with w = 8 < s = 20")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=8, max_subspace_it=6)
    try:
        res = plan.solve_region(torch_cuda.from_numpy(W.start_block(lam.size, 8, 0)).cuda())
        status = rf.RF_OK
    except rf.RfError as e:
        assert e.status == rf.RF_ERR_NOCONV
        res = plan.solve_region(torch_cuda.from_numpy(W.start_block(lam.size, 8, 0)).cuda(),
                                allow_noconv=True)
        status = rf.RF_ERR_NOCONV
    print("status", status, "count", res["count"], "sweeps", res["sweeps"])
    assert res["count"] <= 8
    got = res["lam"]
    if len(got):
        d = np.abs(got[:, None] - inside[None, :]).min(axis=1)
        assert np.all(d <= 1e-8), d.max()
