"""rf_apply_inner_noalloc: G(X) with the library's static work array (no allocation).

Checked through the C ABI against rf_apply_inner (the same kernels on plan buffers)
and the oracle's G, on two calls in a row with the second one smaller, with and
without column chunking, and for the size limit.
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


def _noalloc(torch, plan, X):
    Xd = torch.from_numpy(X).cuda()
    out = torch.full((X.shape[1], X.shape[0]), float("nan"), dtype=torch.complex128,
                     device="cuda").T
    plan.apply_inner_noalloc(Xd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _tridiag_mass_pencil():
    import scipy.sparse as sp
    A, _ = W.convdiff_pencil(16, mass=None)
    n = A.shape[0]
    rng = np.random.default_rng(3)
    d = rng.uniform(0.8, 1.2, n)
    e = 0.1 * rng.uniform(-1, 1, n - 1)
    B = sp.diags([e, d, e], [-1, 0, 1], format="csr", dtype=np.complex128)
    return A, B, 700 + 0.05j, 200.0


@pytest.mark.parametrize("case", ["diagonal_mass", "tridiagonal_mass", "tile256_eight_columns"])
def test_noalloc_matches_apply_inner_twice(rf, torch_cuda, case):
    from oracle import filters
    p, extra = 4, {}
    if case == "diagonal_mass":
        A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=1)
        c, r = 900 + 0.05j, 250.0
    elif case == "tridiagonal_mass":
        A, B, c, r = _tridiag_mass_pencil()
    else:                                        # the 256-thread solve form
        A, B = W.convdiff_pencil(33, mass=(0.5, 1.5), seed=4)
        c, r, p, extra = 3000 + 0.05j, 400.0, 2, dict(tile=256, trsm_cols=8)
    plan = rf.Plan(A, B, c, r, p=p, q=8, w=16, **extra)
    plan.factor_shifts()
    G = filters.InnerOperator(A, B, c, r, p)
    for k, seed in ((16, 2), (5, 3)):            # the second call is smaller
        _say(f"noalloc {case} ncols={k}")
        X = W.start_block(A.shape[0], k, seed=seed)
        Z = _noalloc(torch_cuda, plan, X)
        Zr = plan.apply_inner(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
        e = _colerr(Z, Zr)
        e2 = _colerr(Z, G(X))
        print(f"{case} ncols={k}: vs rf_apply_inner {e.max():.1e}, vs oracle {e2.max():.1e}")
        assert e.max() <= 1e-12 and e2.max() <= 1e-12, (e.max(), e2.max())


def test_noalloc_chunks_at_full_size(rf, torch_cuda):
    # N = 16384, bandwidth 128, p = 4, diagonal B: 2 MiB of work space per column, so
    # 128 columns go in four chunks of 32; then a second, smaller call of 40 columns
    from oracle import filters
    wl = W.convdiff_workload()
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w)
    plan.factor_shifts()
    X = W.start_block(wl.n, 128, seed=11)
    _say("noalloc convdiff128 ncols=128 (chunked)")
    Z = _noalloc(torch_cuda, plan, X)
    Zr = plan.apply_inner(torch_cuda.from_numpy(X).cuda()).cpu().numpy()
    ref = filters.InnerOperator(wl.A, wl.B, wl.c, wl.r, wl.p)(X)
    e, e2 = _colerr(Z, Zr), _colerr(Z, ref)
    print(f"convdiff128 ncols=128: vs rf_apply_inner {e.max():.1e}, vs oracle {e2.max():.1e}")
    assert e.max() <= 1e-12 and e2.max() <= 1e-12
    _say("noalloc convdiff128 ncols=40")
    X2 = W.start_block(wl.n, 40, seed=12)
    Z2 = _noalloc(torch_cuda, plan, X2)
    Zr2 = plan.apply_inner(torch_cuda.from_numpy(X2).cuda()).cpu().numpy()
    e3 = _colerr(Z2, Zr2)
    print(f"convdiff128 ncols=40: vs rf_apply_inner {e3.max():.1e}")
    assert e3.max() <= 1e-12


def test_noalloc_more_columns_than_w(rf, torch_cuda):
    from oracle import filters
    A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=1)
    c, r = 900 + 0.05j, 250.0
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=8)
    plan.factor_shifts()
    X = W.start_block(A.shape[0], 40, seed=5)
    _say("noalloc ncols=40 > w=8")
    Z = _noalloc(torch_cuda, plan, X)
    assert _colerr(Z, filters.InnerOperator(A, B, c, r, 4)(X)).max() <= 1e-12


def test_noalloc_rejects_columns_larger_than_the_array(rf, torch_cuda):
    # diagonal pencil, N = 65536, p = 40: one column needs 65536 * 40 * 32 bytes = 84 MB
    lam = np.linspace(-3, 3, 65536) + 0.5j
    A, B = W.diagonal_pencil(lam)
    _say("noalloc size limit")
    plan = rf.Plan(A, B, 0.0, 1.0, p=40, q=4, w=1, allocator=None)
    X = torch_cuda.zeros((1, 65536), dtype=torch_cuda.complex128, device="cuda").T
    out = torch_cuda.zeros_like(X)
    with pytest.raises(rf.RfError) as ei:
        plan.apply_inner_noalloc(X, out)
    assert ei.value.status == rf.RF_ERR_ARG and "work space" in str(ei.value)
