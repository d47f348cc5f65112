"""GPU parity of the cluster band solve (fused tiles, clusters of nb/16 workgroups per
pole and 16 right-hand sides) against the oracle's G(X) = sum_i w_i K_i^{-1} B X and
against the per-slice solve (solve_form 1) on the same factors.

Shapes: tiles 64 and 128 (and 256, where both forms are the per-slice solve); one, two,
three and many row blocks with a ragged last block (rows past n padded); column counts
that leave a ragged last cluster (1, 17, 40); diagonal B (B X staged by a scaling pass),
B = I, and a general sparse B (B X formed first).  Bar:
max(1e-12, 16 u max cond_2(K_i)) per column against the oracle (both are backward-stable
LU solves of the same systems), and 1e-12 per column between the two device forms.
"""
import sys

import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W

pytestmark = pytest.mark.gpu
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


def _colerr(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def _bar(A, B, c, r, p):
    from oracle import coeffs
    Ad, Bd = A.toarray(), B.toarray()
    poles, _ = coeffs.trapezoid_nodes(c, r, p)
    ck = max(float(np.linalg.cond(z * Bd - Ad)) for z in poles)
    return max(1e-12, 16.0 * U_ROUND * ck)


def _tridiag_mass(n, seed):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.8, 1.2, n)
    e = 0.1 * rng.uniform(-1, 1, n - 1)
    return sp.diags([e, d, e], [-1, 0, 1], format="csr", dtype=np.complex128)


# (name, grid m, tile, mass): N = m^2, bandwidth m
CASES = [
    ("one_block_t64", 7, 64, (0.5, 1.5)),         # N = 49: a single padded block
    ("two_blocks_t64", 10, 64, (0.5, 1.5)),       # N = 100
    ("three_blocks_t128", 18, 128, None),         # N = 324, B = I
    ("seven_blocks_t64_tridiagB", 20, 64, "tri"),  # N = 400, general B
    ("four_blocks_t256", 30, 256, (0.5, 1.5)),    # N = 900 (per-slice form at tile 256)
    ("thirteen_blocks_t128", 40, 128, (0.5, 1.5)),  # N = 1600
]


def _pencil(m, mass):
    if mass == "tri":
        A, _ = W.convdiff_pencil(m, mass=None)
        return A, _tridiag_mass(A.shape[0], 4)
    return W.convdiff_pencil(m, mass=mass, seed=2)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("ncols", [1, 17, 40])
def test_cluster_solve_matches_oracle_and_slices(rf, torch_cuda, case, ncols):
    from oracle import filters
    name, m, tile, mass = CASES[case]
    A, B = _pencil(m, mass)
    n = A.shape[0]
    c, r, p = (m * m * 2.0) + 0.05j, m * m * 0.8, 4
    ncols = min(ncols, n)
    _say(f"cluster solve {name} tile={tile} ncols={ncols}")
    w = max(ncols, 1)
    X = W.start_block(n, ncols, seed=11 + case)
    Xd = torch_cuda.from_numpy(X).cuda()
    cl = rf.Plan(A, B, c, r, p=p, q=4, w=w, tile=tile, tuned=False)
    sl = rf.Plan(A, B, c, r, p=p, q=4, w=w, tile=tile, tuned=False, solve_form=1)
    # the cluster form keeps the fused products beside the factors (tiles 64 and 128)
    if tile <= 128:
        assert cl.device_bytes > sl.device_bytes
    else:
        assert cl.device_bytes == sl.device_bytes
    cl.factor_shifts()
    sl.factor_shifts()
    Zc = cl.apply_inner(Xd).cpu().numpy()
    Zs = sl.apply_inner(Xd).cpu().numpy()
    ref = filters.InnerOperator(A, B, c, r, p)(X)
    ec, es, ecs = _colerr(Zc, ref), _colerr(Zs, ref), _colerr(Zc, Zs)
    bar = _bar(A, B, c, r, p)
    print(f"{name} ncols={ncols}: cluster vs oracle {ec.max():.2e}, slices vs oracle "
          f"{es.max():.2e}, cluster vs slices {ecs.max():.2e} (bar {bar:.1e})")
    assert ec.max() <= bar, (name, ec.max(), bar)
    assert ecs.max() <= max(1e-12, bar), (name, ecs.max())
    # a second application reuses the plan's flags under a new launch epoch
    Zc2 = cl.apply_inner(Xd).cpu().numpy()
    assert np.array_equal(Zc, Zc2)
    cl.close()
    sl.close()


def test_cluster_solve_full_size_columns(rf, torch_cuda):
    # the 128 x 128 workload (tile 128, 128 blocks, 4 poles, 128 columns: 32 clusters of
    # 8 workgroups, the whole device), every column against the per-slice form, and
    # three columns against the oracle
    from oracle import filters
    wl = W.convdiff_workload()
    _say("cluster solve convdiff128 full size")
    X = W.start_block(wl.n, 128, seed=5)
    Xd = torch_cuda.from_numpy(X).cuda()
    cl = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=8, w=128, tuned=False)
    sl = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=8, w=128, tuned=False, solve_form=1)
    cl.factor_shifts()
    sl.factor_shifts()
    Zc = cl.apply_inner(Xd).cpu().numpy()
    Zs = sl.apply_inner(Xd).cpu().numpy()
    e = _colerr(Zc, Zs)
    cols = [0, 63, 127]
    ref = filters.InnerOperator(wl.A, wl.B, wl.c, wl.r, 4)(X[:, cols])
    eo = _colerr(Zc[:, cols], ref)
    print(f"convdiff128: cluster vs slices {e.max():.2e} over 128 columns, vs oracle {eo.max():.2e}")
    assert e.max() <= 1e-12 and eo.max() <= 1e-12, (e.max(), eo.max())
    cl.close()
    sl.close()
