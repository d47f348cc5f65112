"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every block comparison is per column: max over columns c of
||u_c - u*_c|| / ||u*_c||.

Tolerances
----------
* G(X) = sum_i w_i K_i^{-1} B X: both sides are backward-stable banded LU
  solves of the same systems; 1e-12 per column.
* filter_apply on NORMAL pencils (balanced Toeplitz, diagonal): the composite
  method reaches the simple-rule value R_{c,r,pq}(B^{-1}A)Y (Thm. Rcrm) up to the
  outer GMRES tolerance (1e-13 here); 1e-12 per column.
* filter_apply on NON-NORMAL pencils (convection-diffusion): R(B^{-1}A) is a
  function of a matrix whose eigenvector basis X has condition kappa(X) of 1e4 to
  1e5, so any floating-point evaluation of it -- the oracle's two direct ones
  (band LU, dense LAPACK) included -- is only defined to about
  kappa(X) u max(||y_c||, ||u*_c||).  The bar is that times 16, over ||u*_c||, plus
  the oracle's own spread (band LU vs dense solves) per column, all computed densely
  in the test, and the measured error is printed beside kappa(X) u and cond(K_i).
* eigenpairs: |dlambda|/|lambda| <= 1e-10 over a minimum-cost assignment of the
  eigenvalues, and e_i <= 1e-10 (eq. rel-error) re-evaluated by the oracle.
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


U_ROUND = np.finfo(np.float64).eps / 2          # unit roundoff 1.1e-16


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _colerr(a, b):
    """per-column relative errors ||a_c - b_c|| / ||b_c||"""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def _match_rel(lam, ref):
    """|lambda_i - ref_pi(i)| / |ref_pi(i)| over the minimum-cost assignment pi of
    the computed eigenvalues to the reference ones (equal counts)"""
    from scipy.optimize import linear_sum_assignment
    lam, ref = np.asarray(lam), np.asarray(ref)
    assert len(lam) == len(ref), (len(lam), len(ref))
    cost = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(cost)
    return cost[r, c] / np.abs(ref[c])


_DENSE = {}


def _dense_bar(name, A, B, c, r, p, q, Y):
    """For a small non-normal pencil: (oracle block, bar per column, kappa(X) u, max
    cond(K_i), oracle spread).  The oracle's simple rule with pq poles is evaluated
    twice, by its band LU and by dense LAPACK solves; their per-column difference is
    the oracle's own rounding spread.  kappa(X) is the condition number of the
    eigenvector matrix of B^{-1} A.  A backward-stable evaluation of R(B^{-1}A) y
    perturbs it by a matrix of norm about kappa(X) u times the size of the filter, so
    its error scales with the larger of ||y|| and ||R y|| (R damps the columns of a
    nearly invariant block outside the disk and, the pencil being non-normal, can also
    amplify a column): the bar on ||u_c - u*_c|| / ||u*_c|| is
    16 kappa(X) u max(||y_c||, ||u*_c||) / ||u*_c|| + spread_c."""
    from oracle import coeffs, filters
    key = (name, p, q, Y.shape[1])
    if key not in _DENSE:
        Ad, Bd = A.toarray(), B.toarray()
        poles, wts = coeffs.trapezoid_nodes(c, r, p * q)
        dense = sum(wi * np.linalg.solve(z * Bd - Ad, Bd @ Y) for z, wi in zip(poles, wts))
        band = filters.simple_filter(A, B, c, r, p * q, Y)
        _, X = np.linalg.eig(np.linalg.solve(Bd, Ad))
        kx = np.linalg.cond(X) * U_ROUND
        ip, _ = coeffs.trapezoid_nodes(c, r, p)
        ck = max(np.linalg.cond(z * Bd - Ad) for z in ip)
        spread = _colerr(dense, band)
        ny, nu = np.linalg.norm(Y, axis=0), np.linalg.norm(band, axis=0)
        scale = np.maximum(ny, nu) / nu
        _DENSE[key] = (band, 16.0 * kx * scale + spread, kx, ck, spread.max())
    return _DENSE[key]


_GBAR = {}


def _g_bar(name, A, B, c, r, p):
    """Bar for G(X) against the oracle: both sides solve with backward-stable band
    LUs of the K_i, so they agree to about cond(K_i) u: max(1e-12, 16 u max cond_2(K_i)),
    the condition numbers computed densely."""
    from oracle import coeffs
    if name not in _GBAR:
        Ad, Bd = A.toarray(), B.toarray()
        poles, _ = coeffs.trapezoid_nodes(c, r, p)
        ck = max(float(np.linalg.cond(z * Bd - Ad)) for z in poles)
        _GBAR[name] = max(1e-12, 16.0 * U_ROUND * ck)
    return _GBAR[name]


def _to_host(X):
    return X.cpu().numpy()


def _pencils():
    out = []
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    out.append(("toeplitz2000", wl.A, wl.B, wl.c, wl.r))
    A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=1)          # N=400, kl=20: ragged tail
    out.append(("convdiff20", A, B, 900 + 0.05j, 250.0))
    A, B = W.convdiff_pencil(33, mass=None)                          # B = I, N=1089, kl=33
    out.append(("convdiff33_I", A, B, 3000 + 0.05j, 400.0))
    # non-diagonal B (tridiagonal mass): exercises the general CSR path of B X
    A, _ = W.convdiff_pencil(16, mass=None)
    import scipy.sparse as sp
    N = A.shape[0]
    rng = np.random.default_rng(3)
    d = rng.uniform(0.8, 1.2, N)
    e = 0.1 * rng.uniform(-1, 1, N - 1)
    Bt = sp.diags([e, d, e], [-1, 0, 1], format="csr", dtype=np.complex128)
    out.append(("convdiff16_tridiagB", A, Bt, 700 + 0.05j, 200.0))
    return out


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("ncols", [1, 7, 32])
def test_inner_apply_matches_oracle(rf, torch_cuda, case, ncols):
    from oracle import filters
    name, A, B, c, r = _pencils()[case]
    _say(f"inner_apply {name} ncols={ncols}")
    p = 4
    plan = rf.Plan(A, B, c, r, p=p, q=4, w=32)
    plan.factor_shifts()
    X = W.start_block(A.shape[0], ncols, seed=7)
    Z = _to_host(plan.apply_inner(torch_cuda.from_numpy(X).cuda()))
    ref = filters.InnerOperator(A, B, c, r, p)(X)
    e = _colerr(Z, ref)
    assert e.max() <= 1e-12, (name, e.max())


@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("ncols", [1, 7, 32])
def test_adjoint_inner_apply_matches_oracle(rf, torch_cuda, case, ncols):
    # the adjoint plan solves with the conjugate transposes of the plan's factors
    # (K_i^H = U_i^H L_i^H P_i^T); its G must equal the oracle's G of the adjoint pencil
    # (A^H, B^H) over the mirrored disk, factorized on its own
    from oracle import filters
    name, A, B, c, r = _pencils()[case]
    _say(f"adjoint inner_apply {name} ncols={ncols}")
    plan = rf.Plan(A, B, c, r, p=4, q=4, w=32)
    plan.factor_shifts()
    adj = plan.adjoint()
    adj.factor_shifts()
    X = W.start_block(A.shape[0], ncols, seed=9)
    Z = _to_host(adj.apply_inner(torch_cuda.from_numpy(X).cuda()))
    AH, BH = A.conj().T.tocsr(), B.conj().T.tocsr()
    ref = filters.InnerOperator(AH, BH, np.conj(c), r, 4)(X)
    e = _colerr(Z, ref)
    bar = _g_bar(name, A, B, c, r, 4)
    print(f"adjoint G {name} ncols={ncols}: per-column error {e.max():.2e} (bar {bar:.1e})")
    assert e.max() <= bar, (name, e.max())
    # no factorization of its own: it holds only the transposed tiles and row orders
    assert adj.device_bytes < plan.device_bytes
    adj.close()
    plan.close()


@pytest.mark.parametrize("tile", [16, 32, 64, 128, 256])
def test_adjoint_inner_apply_tiles(rf, torch_cuda, tile):
    from oracle import filters
    A, B = W.convdiff_pencil(12, mass=(0.5, 1.5), seed=5)           # kl = 12, N = 144
    c, r = 300 + 0.05j, 100.0
    X = W.start_block(A.shape[0], 13, seed=2)
    ref = filters.InnerOperator(A.conj().T.tocsr(), B.conj().T.tocsr(), np.conj(c), r, 3)(X)
    _say(f"adjoint inner_apply tile={tile}")
    plan = rf.Plan(A, B, c, r, p=3, q=4, w=16, tile=tile)
    adj = plan.adjoint()
    with pytest.raises(rf.RfError) as ei:            # the plan has no factors yet
        adj.factor_shifts()
    assert ei.value.status == rf.RF_ERR_STATE
    plan.factor_shifts()
    adj.factor_shifts()
    Z = _to_host(adj.apply_inner(torch_cuda.from_numpy(X).cuda()))
    assert _colerr(Z, ref).max() <= 1e-12, (tile, _colerr(Z, ref).max())
    adj.close()
    plan.close()


def test_inner_apply_tile_override_and_column_slices(rf, torch_cuda):
    from oracle import filters
    A, B = W.convdiff_pencil(12, mass=(0.5, 1.5), seed=5)           # kl = 12
    X = W.start_block(A.shape[0], 16, seed=2)
    ref = filters.InnerOperator(A, B, 300 + 0.05j, 100.0, 3)(X)
    for tile, cols in [(16, 1), (32, 2), (64, 4), (128, 8)]:
        _say(f"inner_apply tile={tile} trsm_cols={cols}")
        plan = rf.Plan(A, B, 300 + 0.05j, 100.0, p=3, q=4, w=16, tile=tile, trsm_cols=cols)
        plan.factor_shifts()
        Z = _to_host(plan.apply_inner(torch_cuda.from_numpy(X).cuda()))
        assert _colerr(Z, ref).max() <= 1e-12, (tile, cols)


@pytest.mark.parametrize("tile", [64, 128])
def test_inner_apply_slice_width_agreement(rf, torch_cuda, tile):
    # each right-hand side of a solve workgroup accumulates the same tile elements in
    # the same order whatever the slice width, so 1, 2 and 4 columns per workgroup
    # (the v-prefetching products at 1 and 2, the plain ones at 4) agree to rounding
    # (not bit for bit: the compiler may contract the complex weight and mass products
    # into fused multiply-adds differently in each instantiation)
    A, B = W.convdiff_pencil(33, mass=(0.5, 1.5), seed=4)           # N = 1089: ragged last block
    X = torch_cuda.from_numpy(W.start_block(A.shape[0], 13, seed=5)).cuda()   # ragged slices
    out = []
    for cols in (1, 2, 4):
        _say(f"inner_apply tile={tile} trsm_cols={cols} (agreement across slice widths)")
        plan = rf.Plan(A, B, 3000 + 0.05j, 400.0, p=3, q=4, w=24, tile=tile, trsm_cols=cols)
        plan.factor_shifts()
        out.append(_to_host(plan.apply_inner(X)))
        plan.close()
    d = [_colerr(out[i], out[0]).max() for i in (1, 2)]
    _say(f"  relative differences vs one column per workgroup: {d[0]:.1e}, {d[1]:.1e}")
    assert max(d) <= 1e-14, d


@pytest.mark.parametrize("precision", [0, 1])
def test_inner_apply_tile_256(rf, torch_cuda, precision):
    # the largest tile: 16-column factorization sub-steps (LDS), four rows per solve
    # thread; N = 1089 gives 5 block steps with a ragged last block
    from oracle import filters
    A, B = W.convdiff_pencil(33, mass=(0.5, 1.5), seed=4)           # kl = 33
    X = W.start_block(A.shape[0], 24, seed=3)
    ref = filters.InnerOperator(A, B, 3000 + 0.05j, 400.0, 2)(X)
    for cols in (1, 2, 4):
        _say(f"inner_apply tile=256 trsm_cols={cols} precision={precision}")
        plan = rf.Plan(A, B, 3000 + 0.05j, 400.0, p=2, q=4, w=24, tile=256, trsm_cols=cols,
                       precision=precision)
        plan.factor_shifts()
        Z = _to_host(plan.apply_inner(torch_cuda.from_numpy(X).cuda()))
        e = _colerr(Z, ref).max()
        assert e <= (1e-12 if precision == 0 else 1e-5), (cols, e)
        plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_inner_apply_tile_256_eight_columns(rf, torch_cuda, precision):
    # eight right-hand sides per solve workgroup at tile 256 (complex128: 256 threads,
    # the forward window in three nb-row buffers in turn; complex64: 512 threads), against
    # the oracle and against four columns per workgroup.  In complex128 four columns split
    # each row's inner products over 8 lanes instead of 4, so the two agree to rounding;
    # in complex64 the split is the same.  21 columns give a ragged last slice; N = 1089
    # gives five block steps (the buffers go round more than once) with a ragged last block.
    from oracle import filters
    A, B = W.convdiff_pencil(33, mass=(0.5, 1.5), seed=4)           # kl = 33
    X = W.start_block(A.shape[0], 21, seed=6)
    ref = filters.InnerOperator(A, B, 3000 + 0.05j, 400.0, 2)(X)
    out = {}
    for cols in (4, 8):
        _say(f"inner_apply tile=256 trsm_cols={cols} precision={precision} (21 columns)")
        plan = rf.Plan(A, B, 3000 + 0.05j, 400.0, p=2, q=4, w=24, tile=256, trsm_cols=cols,
                       precision=precision)
        plan.factor_shifts()
        out[cols] = _to_host(plan.apply_inner(torch_cuda.from_numpy(X).cuda()))
        plan.close()
    e = _colerr(out[8], ref).max()
    d = _colerr(out[8], out[4]).max()
    _say(f"  eight columns per workgroup: {e:.1e} from the oracle, {d:.1e} from four")
    assert e <= (1e-12 if precision == 0 else 1e-5), e
    assert d <= (1e-14 if precision == 0 else 1e-6), d


def test_factorization_graph_replays_match_eager(rf, torch_cuda):
    # on a non-null stream rf_factor_shifts records its launch sequence in a HIP graph
    # once and replays it; every replay, with eager work and synchronizations of the
    # program in between, must give the factors of plain launches bit for bit
    A, B = W.convdiff_pencil(24, mass=(0.5, 1.5), seed=4)           # N = 576, 19 block steps
    c, r = 1500 + 0.05j, 300.0
    X = torch_cuda.from_numpy(W.start_block(A.shape[0], 16, seed=2)).cuda()
    side = torch_cuda.cuda.Stream()
    _say("factorization graph replays vs eager launches")
    eager = rf.Plan(A, B, c, r, p=4, q=8, w=16, no_graph=1, stream=side)
    eager.factor_shifts()
    with torch_cuda.cuda.stream(side):
        ref = eager.apply_inner(X).cpu().numpy()
    graph = rf.Plan(A, B, c, r, p=4, q=8, w=16, stream=side)
    for rep in range(4):
        graph.factor_shifts()
        with torch_cuda.cuda.stream(side):
            Z = graph.apply_inner(X).cpu().numpy()
        assert np.array_equal(Z, ref), rep
        # eager work of the program between replays
        Y = torch_cuda.randn(2048, 2048, device="cuda") @ torch_cuda.randn(2048, 2048, device="cuda")
        torch_cuda.cuda.synchronize()
        assert torch_cuda.isfinite(Y).all()
        eager.factor_shifts()
    graph.close()
    eager.close()


def test_pole_on_eigenvalue_is_reported_singular(rf, torch_cuda):
    # diagonal pencil with an eigenvalue exactly at a trapezoidal pole
    lam = np.linspace(-3, 3, 64) + 0.0j
    c, r, p = 0.0, 1.0, 4
    pole = c + r * np.exp(1j * np.pi / p)
    lam[10] = pole
    A, B = W.diagonal_pencil(lam)
    _say("singular pole")
    plan = rf.Plan(A, B, c, r, p=p, q=4, w=8)
    with pytest.raises(rf.RfError) as ei:
        plan.factor_shifts()
    assert ei.value.status == rf.RF_ERR_SINGULAR


@pytest.mark.parametrize("q", [4, 8, 3])
def test_filter_apply_matches_simple_rule(rf, torch_cuda, q):
    # balanced Toeplitz (normal): the composite filter equals the simple rule with pq
    # poles (Thm. Rcrm) to 1e-12 per column
    from oracle import filters
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    _say(f"filter_apply toeplitz2000 q={q}")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=q, w=32, gmres_tol=1e-13)
    plan.factor_shifts()
    Y = W.start_block(wl.n, 32, seed=3)
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    ref = filters.simple_filter(wl.A, wl.B, wl.c, wl.r, 4 * q, Y)
    assert info["converged"]
    e = _colerr(_to_host(U), ref)
    print(f"toeplitz2000 q={q}: per-column filter error max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() <= 1e-12, e.max()


@pytest.mark.parametrize("q", [8, 16])
def test_filter_apply_diagonal_pencil_closed_form(rf, torch_cuda, q):
    # diagonal pencil A = diag(a_j), B = diag(b_j) (normal): the filter is
    # diag(1 / (1 + ((a_j/b_j - c)/r)^(pq))) Y exactly (Lemma compact with eq. pwtp),
    # written out here; the oracle's simple rule is checked too
    from oracle import filters
    rng = np.random.default_rng(5)
    lam = rng.uniform(-3, 3, 800) + 1j * rng.uniform(-1, 1, 800)
    bd = rng.uniform(0.5, 1.5, 800)
    A, B = W.diagonal_pencil(lam, bd)
    c, r, p = 0.2 + 0.1j, 1.0, 4
    _say(f"filter_apply diagonal800 q={q}")
    plan = rf.Plan(A, B, c, r, p=p, q=q, w=32, gmres_tol=1e-13)
    plan.factor_shifts()
    Y = W.start_block(800, 32, seed=3)
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    assert info["converged"]
    closed = (1.0 / (1.0 + ((lam - c) / r) ** (p * q)))[:, None] * Y
    e = _colerr(_to_host(U), closed)
    e2 = _colerr(_to_host(U), filters.simple_filter(A, B, c, r, p * q, Y))
    print(f"diagonal800 q={q}: per-column error vs closed form {e.max():.2e}, vs oracle {e2.max():.2e}")
    assert e.max() <= 1e-12 and e2.max() <= 1e-12, (e.max(), e2.max())


def _nonnormal_filter_case(rf, torch_cuda, name, A, B, c, r, p, q, w, **opts):
    Y = W.start_block(A.shape[0], w, seed=8)
    ref, bar, kx, ck, spread = _dense_bar(name, A, B, c, r, p, q, Y)
    plan = rf.Plan(A, B, c, r, p=p, q=q, w=w, gmres_tol=1e-13, **opts)
    plan.factor_shifts()
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    assert info["converged"]
    e = _colerr(_to_host(U), ref)
    print(f"{name}: per-column filter error max {e.max():.2e} median {np.median(e):.2e}; "
          f"kappa(X) u {kx:.2e}, oracle spread {spread:.2e}, max cond(K_i) {ck:.2e}")
    assert np.all(e <= bar), (e / bar).max()
    return e


@pytest.mark.parametrize("subblock", [8, 16, 32])
def test_filter_apply_convdiff_random_mass(rf, torch_cuda, subblock):
    A, B = W.convdiff_pencil(24, mass=(0.5, 1.5), seed=4)           # N=576, kl=24
    _say(f"filter_apply convdiff24 subblock={subblock}")
    _nonnormal_filter_case(rf, torch_cuda, "convdiff24_mass", A, B, 1500 + 0.05j, 300.0, 4, 8, 32,
                           subblock=subblock)


def test_filter_apply_convdiff_identity_mass(rf, torch_cuda):
    # constant-coefficient convection-diffusion, B = I: similar to a symmetric matrix
    # through a diagonal scaling, but that scaling has condition 1e5 at n = 33
    A, B = W.convdiff_pencil(33, mass=None)
    _say("filter_apply convdiff33 B = I")
    _nonnormal_filter_case(rf, torch_cuda, "convdiff33_I", A, B, 3000 + 0.05j, 400.0, 4, 8, 32)


def test_solve_region_toeplitz_closed_form(rf, torch_cuda):
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    _say("solve_region toeplitz2000")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=32, expected_count=20)
    Y0 = torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda()
    res = plan.solve_region(Y0)
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    assert res["converged"] and res["count"] == len(inside) == 20
    rel = _match_rel(res["lam"], inside)
    print(f"toeplitz2000: max |dlambda|/|lambda| {rel.max():.2e}")
    assert rel.max() <= 1e-10, rel.max()
    assert res["err"].max() <= 1e-10


def test_solve_region_literal_toeplitz(rf, torch_cuda):
    # the literal Toeplitz pencil (a = 0, b = 1, c = 0.5 e^{i pi/3}) is exponentially
    # non-normal: its eigenvalue condition numbers grow like (|b|/|c|)^{(n-1)/2}.  At
    # n = 40 (kappa ~ 1e5..1e6, from dense left and right eigenvectors) the eigenvalues
    # are defined in FP64 and the solver must find them all, each within the first-order
    # bound kappa * residual norm of its returned pair (a pair with e <= 1e-10 is not
    # closer than that); at n = 2000 no FP64 method can find them (sigma_min(z I - A) ~
    # 1e-265 near the disk): the pairs returned are pseudo-eigenpairs whose residuals meet
    # the bar, and their distance to the closed form is printed as measured
    from oracle import hsrr, sensitivity
    from scipy.optimize import linear_sum_assignment
    wl = W.toeplitz_workload(n=40, balanced=False, w=8, count=4, c=0.3 + 0.2j)
    exact = W.toeplitz_eigs(40, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    _say("solve_region literal toeplitz n=40")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=8, expected_count=len(inside))
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(40, 8, 0)).cuda())
    assert res["converged"] and res["count"] == len(inside)
    lam_d, X_d, Y_d = sensitivity.dense_left_right(wl.A, wl.B)
    lam_d, X_d, Y_d = sensitivity.select(lam_d, X_d, Y_d, inside)
    kap = np.linalg.norm(X_d, axis=0) * np.linalg.norm(Y_d, axis=0) / np.abs(
        np.einsum("ij,ij->j", Y_d.conj(), X_d))
    cost = np.abs(res["lam"][:, None] - inside[None, :])
    r_, c_ = linear_sum_assignment(cost)
    e = hsrr.rel_errors(wl.A, wl.B, res["lam"], _to_host(res["X"]), wl.c, wl.r)
    rn = e * (abs(wl.c) + wl.r)                       # residual norms of the unit vectors (B = I)
    bound = kap[c_] * rn[r_] + 1e-13 * np.abs(inside[c_])
    print(f"literal toeplitz n=40: {len(inside)} eigenvalues, kappa {kap.min():.1e}..{kap.max():.1e}, "
          f"max |dlambda|/|lambda| {(cost[r_, c_] / np.abs(inside[c_])).max():.2e}, max ratio to "
          f"kappa * residual {(cost[r_, c_] / bound).max():.2f}")
    assert e.max() <= 1e-10 and np.all(cost[r_, c_] <= bound)
    wl = W.toeplitz_workload(n=2000, balanced=False, w=32, count=20)
    _say("solve_region literal toeplitz n=2000")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=32)
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda(),
                            allow_noconv=True)
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    e = hsrr.rel_errors(wl.A, wl.B, res["lam"], _to_host(res["X"]), wl.c, wl.r)
    d = (np.abs(res["lam"][:, None] - exact[None, :]).min(axis=1) if res["count"] else np.zeros(0))
    print(f"literal toeplitz n=2000: {res['count']} pairs returned (20 closed-form eigenvalues in the "
          f"disk), sweeps {res['sweeps']}, max residual {e.max() if len(e) else 0:.1e}, distance to the "
          f"closed form {d.min() if len(d) else float('nan'):.1e}..{d.max() if len(d) else float('nan'):.1e}")
    assert np.all(e <= 1e-10)


def test_solve_region_small_convdiff_vs_oracle(rf, torch_cuda):
    from oracle import hsrr, solver
    import scipy.linalg as sl
    n = 20
    A, B = W.convdiff_pencil(n, mass=(0.5, 1.5), seed=6)
    lam_all = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam_all.real)[150] + 0.05j
    r = W.midgap_radius(lam_all, c, 12)
    Y0 = W.start_block(n * n, 16, 1)
    _say("solve_region convdiff20")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=16, expected_count=12)
    res = plan.solve_region(torch_cuda.from_numpy(Y0).cuda())
    ref = solver.solve_region(A, B, c, r, 4, 8, Y0, s_expected=12)
    assert res["count"] == len(ref.lam) == 12
    rel = _match_rel(res["lam"], ref.lam)
    print(f"convdiff20: max |dlambda|/|lambda| {rel.max():.2e}")
    assert rel.max() <= 1e-10, rel.max()
    # residuals re-evaluated by the oracle's definition on the returned vectors
    e = hsrr.rel_errors(A, B, res["lam"], _to_host(res["X"]), c, r)
    assert e.max() <= 1e-10


@pytest.mark.parametrize("subblock", [8, 16])
def test_filter_apply_on_converged_ritz_vectors(rf, torch_cuda, subblock):
    # After solve_region the Ritz block is nearly invariant; the outer solves must
    # still converge and the filter must still match the simple rule.
    from oracle import filters
    n = 24
    A, B = W.convdiff_pencil(n, mass=(0.5, 1.5), seed=3)
    import scipy.linalg as sl
    lam = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam.real)[200] + 0.05j
    r = W.midgap_radius(lam, c, 24)
    _say(f"filter on ritz vectors subblock={subblock}")
    plan = rf.Plan(A, B, c, r, p=4, q=8, w=32, subblock=subblock, gmres_tol=1e-12,
                   max_krylov_blocks=60, expected_count=24)
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(n * n, 32, 0)).cuda())
    Xr = res["all_X"]
    U, info = plan.filter_apply(Xr, allow_noconv=True)
    ref, bar, kx, ck, spread = _dense_bar(f"ritz{subblock}", A, B, c, r, 4, 8, _to_host(Xr))
    e = _colerr(_to_host(U), ref)
    print(f"ritz block subblock={subblock}: krylov steps {info['krylov_steps']}, max residual "
          f"{info['max_residual']:.1e}, per-column filter error max {e.max():.2e}; kappa(X) u "
          f"{kx:.2e}, oracle spread {spread:.2e}, max cond(K_i) {ck:.2e}")
    assert info["converged"], info
    assert np.all(e <= bar), (e / bar).max()


# ---------------------------------------------------------------------------
# full size: the 128 x 128 convection-diffusion workload the benchmark times
# (N = 16384, bandwidth 128, p = 4, q = 8, w = 128)
# ---------------------------------------------------------------------------
def _golden_convdiff128():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "convdiff128_eigs.txt")
    lam, err = [], []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        re_, im_, e_ = (float(x) for x in line.split())
        lam.append(complex(re_, im_))
        err.append(e_)
    return np.array(lam), np.array(err)


@pytest.fixture(scope="module")
def convdiff128(rf, torch_cuda):
    wl = W.convdiff_workload()
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w,
                   expected_count=wl.s_expected, gmres_tol=1e-13)
    plan.factor_shifts()
    return wl, plan


def test_full_size_inner_apply_all_columns(rf, torch_cuda, convdiff128):
    # G on all 128 columns in the benchmark's launch shape, every column checked
    # against the oracle's G (four band LUs and solves, about 7 s on one core)
    from oracle import filters
    wl, plan = convdiff128
    _say("convdiff128 apply_inner, 128 columns")
    X = W.start_block(wl.n, wl.w, seed=11)
    Z = _to_host(plan.apply_inner(torch_cuda.from_numpy(X).cuda()))
    ref = filters.InnerOperator(wl.A, wl.B, wl.c, wl.r, wl.p)(X)
    e = _colerr(Z, ref)
    print(f"convdiff128 G: per-column error max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() <= 1e-12, e.max()


def test_full_size_filter_apply_all_columns(rf, torch_cuda, convdiff128):
    # one composite filter application on the 128-column start block, every column
    # against the oracle's simple rule with pq = 32 poles, stored as a 128-vector
    # Gaussian sketch of each column (tests/golden/make_convdiff128_filter.py).  The
    # pencil is non-normal: the filtered columns lie in the span of the eigenvectors
    # inside the disk, whose eigenvalue condition numbers kappa_B reach 1.2e4
    # (tests/golden/convdiff128_cond.txt), so the bar is 16 max(kappa_B) u per column
    # as on the small non-normal pencils (where kappa(X) is computed densely).
    import os
    wl, plan = convdiff128
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g = np.load(os.path.join(here, "convdiff128_filter_sketch.npz"))
    kappa = np.loadtxt(os.path.join(here, "convdiff128_cond.txt"))[:, 2].max()
    assert int(g["y_seed"]) == wl.seed and int(g["k"]) == wl.p * wl.q
    _say("convdiff128 filter_apply, 128 columns")
    Y = W.start_block(wl.n, wl.w, wl.seed)
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    assert info["converged"], info
    Uh = _to_host(U)
    S = W.start_block(wl.n, 128, int(g["sketch_seed"]))
    sk = S.conj().T @ Uh
    e = np.linalg.norm(sk - g["sketch"], axis=0) / np.linalg.norm(g["sketch"], axis=0)
    nrm = np.abs(np.linalg.norm(Uh, axis=0) / g["norms"] - 1.0)
    bar = 16.0 * kappa * U_ROUND
    print(f"convdiff128 filter: per-column sketched error max {e.max():.2e} median "
          f"{np.median(e):.2e}, column-norm deviation max {nrm.max():.1e}, krylov steps "
          f"{info['krylov_steps']}; 16 max(kappa_B) u = {bar:.2e}")
    assert e.max() <= bar and nrm.max() <= bar, (e.max(), nrm.max(), bar)


def test_full_size_solve_region_matches_oracle(rf, torch_cuda, convdiff128):
    # eigenpairs of the benchmark workload vs the oracle's own full Alg. composite run
    # (tests/golden/convdiff128_eigs.txt, written by tests/golden/make_convdiff128.py)
    from oracle import hsrr
    from scipy.optimize import linear_sum_assignment
    wl, plan = convdiff128
    ref_lam, ref_err = _golden_convdiff128()
    _say("convdiff128 solve_region")
    Y0 = torch_cuda.from_numpy(W.start_block(wl.n, wl.w, wl.seed)).cuda()
    res = plan.solve_region(Y0)
    assert res["converged"]
    assert res["count"] == len(ref_lam) == wl.s_expected
    cost = np.abs(res["lam"][:, None] - ref_lam[None, :])
    r, c = linear_sum_assignment(cost)
    rel = cost[r, c] / np.abs(ref_lam[c])
    print("max |dlambda|/|lambda|", rel.max(), "median", np.median(rel))
    assert rel.max() <= 1e-10, rel.max()
    e = hsrr.rel_errors(wl.A, wl.B, res["lam"], _to_host(res["X"]), wl.c, wl.r)
    print("max residual (oracle's definition)", e.max())
    assert e.max() <= 1e-10


# ---------------------------------------------------------------------------
# Alg. composite2: no subspace iteration, outer node count doubling on one basis
# ---------------------------------------------------------------------------
def test_solve_region_adaptive_small_convdiff_vs_oracle(rf, torch_cuda):
    from oracle import hsrr, solver
    import scipy.linalg as sl
    n = 20
    A, B = W.convdiff_pencil(n, mass=(0.5, 1.5), seed=6)
    lam_all = sl.eigvals(A.toarray(), B.toarray())
    c = np.sort(lam_all.real)[150] + 0.05j
    r = W.midgap_radius(lam_all, c, 12)
    Y0 = W.start_block(n * n, 16, 1)
    _say("solve_region_adaptive convdiff20")
    plan = rf.Plan(A, B, c, r, p=4, q=4, q_max=64, w=16, expected_count=12, gmres_tol=1e-13)
    res = plan.solve_region_adaptive(torch_cuda.from_numpy(Y0).cuda())
    ref = solver.solve_region_adaptive(A, B, c, r, 4, 4, 64, Y0, s_expected=12)
    print("levels", res["sweeps"], ref.sweeps, "basis depth", res["krylov_steps"])
    assert res["converged"] and ref.converged
    assert res["count"] == len(ref.lam) == 12
    assert res["sweeps"] == ref.sweeps
    rel = _match_rel(res["lam"], ref.lam)
    assert rel.max() <= 1e-10, rel.max()
    e = hsrr.rel_errors(A, B, res["lam"], _to_host(res["X"]), c, r)
    assert e.max() <= 1e-10
    # the plan's own rule is back in place: filter_apply still matches the simple rule
    from oracle import filters
    Y = W.start_block(n * n, 16, seed=3)
    U, info = plan.filter_apply(torch_cuda.from_numpy(Y).cuda())
    ref, bar, kx, ck, spread = _dense_bar("convdiff20_ad", A, B, c, r, 4, 4, Y)
    assert np.all(_colerr(_to_host(U), ref) <= bar)


def test_solve_region_adaptive_toeplitz_closed_form(rf, torch_cuda):
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    _say("solve_region_adaptive toeplitz2000")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, q_max=64, w=32, expected_count=20)
    res = plan.solve_region_adaptive(torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda())
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    assert res["converged"] and res["count"] == len(inside) == 20
    rel = _match_rel(res["lam"], inside)
    assert rel.max() <= 1e-10, rel.max()
    assert res["err"].max() <= 1e-10


# ---------------------------------------------------------------------------
# the paper's circuit workload (App. B), n_x = 10: k1 = k2 = 8, n_col = 24
# ---------------------------------------------------------------------------
def test_solve_region_circuit10_vs_dense(rf, torch_cuda):
    import scipy.linalg as sl
    from oracle import hsrr
    wl = W.circuit_workload()
    _say("solve_region circuit10 (p = q = 8, w = 24)")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=wl.q, w=wl.w, expected_count=wl.s_expected)
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(wl.n, wl.w, 0)).cuda())
    w = sl.eigvals(wl.A.toarray(), wl.B.toarray())
    w = w[np.isfinite(w)]
    inside = w[np.abs(w - wl.c) < wl.r]
    assert res["converged"] and res["count"] == len(inside) == wl.s_expected
    rel = _match_rel(res["lam"], inside)
    assert rel.max() <= 1e-10, rel.max()
    e = hsrr.rel_errors(wl.A, wl.B, res["lam"], _to_host(res["X"]), wl.c, wl.r)
    assert e.max() <= 1e-10


def test_solve_region_adaptive_circuit10_vs_dense(rf, torch_cuda):
    import scipy.linalg as sl
    wl = W.circuit_workload()
    _say("solve_region_adaptive circuit10 (p = 8, q = 2 .. 16)")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=wl.p, q=2, w=wl.w, expected_count=wl.s_expected,
                   q_max=16)
    res = plan.solve_region_adaptive(torch_cuda.from_numpy(W.start_block(wl.n, wl.w, 0)).cuda())
    w = sl.eigvals(wl.A.toarray(), wl.B.toarray())
    w = w[np.isfinite(w)]
    inside = w[np.abs(w - wl.c) < wl.r]
    assert res["converged"] and res["count"] == len(inside)
    rel = _match_rel(res["lam"], inside)
    assert rel.max() <= 1e-10, rel.max()


def test_solve_region_sweep_cap_returns_noconv_with_results(rf, torch_cuda):
    # one sweep allowed and no expected count: the stopping rule cannot be met (it needs
    # two equal counts), so the call reports RF_ERR_NOCONV with the sweep's pairs filled in
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    _say("solve_region toeplitz2000, sweep cap 1")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=32, max_subspace_it=1)
    with pytest.raises(rf.RfError) as e:
        plan.solve_region(torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda())
    assert e.value.status == rf.RF_ERR_NOCONV
    res = plan.solve_region(torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda(),
                            allow_noconv=True)
    assert res["sweeps"] == 1 and not res["converged"]
    exact = W.toeplitz_eigs(wl.n, 0, 1, W.TOEPLITZ_C)
    inside = exact[np.abs(exact - wl.c) < wl.r]
    # after one sweep the filtered pairs (inside D, e < tau_g) are the 20 eigenvalues, to
    # the accuracy their residuals allow (the matrix is normal: |dlambda| <= residual)
    filt = (res["flags"] & 3) == 3
    assert filt.sum() == len(inside)
    lam = res["all_lam"][filt]
    d = np.abs(lam[:, None] - inside[None, :]).min(axis=1)
    resid = res["all_err"][filt] * (abs(wl.c) + wl.r)
    assert np.all(d <= 2.0 * resid + 1e-12)


def test_solve_region_repeatable_and_independent_of_previous_calls(rf, torch_cuda):
    # the plan keeps no state between calls except the factors: two calls with the same
    # start block give the same pairs, bit for bit
    wl = W.toeplitz_workload(n=2000, w=32, count=20)
    _say("solve_region toeplitz2000 twice")
    plan = rf.Plan(wl.A, wl.B, wl.c, wl.r, p=4, q=4, w=32, expected_count=20)
    Y0 = torch_cuda.from_numpy(W.start_block(wl.n, 32, 0)).cuda()
    r1 = plan.solve_region(Y0)
    r2 = plan.solve_region(Y0)
    assert np.array_equal(r1["all_lam"], r2["all_lam"])
    assert np.array_equal(r1["all_err"], r2["all_err"])
