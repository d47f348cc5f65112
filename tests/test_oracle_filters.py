"""Pins of the oracle's filters against spectral closed forms.

For a diagonalizable pencil with B^{-1}A = X Lambda X^{-1}, eq.
discretizedCIoperator together with Lemma compact gives
    R_{c,r,k}(B^{-1}A) Y = X diag(1/(1 + ((lambda_j - c)/r)^k)) X^{-1} Y.
Three pencils have X in closed form: diagonal pencils, the balanced
tridiagonal Toeplitz pencil (X = the orthonormal DST-I matrix), and the
constant-coefficient upwind convection-diffusion operator with B = I
(X = a Kronecker product of diagonally scaled DST-I matrices).

The composite path (inner direct solves + per-column multi-shift GMRES) must
reproduce the simple rule with pq poles (Thm. Rcrm, Sec. 5).
"""
import numpy as np
import pytest

from oracle import coeffs, filters, gmres
from paper_2310_18043_amd import workloads as W

RNG = np.random.default_rng(11)


def _compact(z, c, r, k):
    return 1.0 / (1.0 + ((z - c) / r) ** k)


def _dst(n):
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k", [4, 16, 32])
def test_simple_filter_diagonal_pencil(k):
    n, c, r = 60, 0.5 + 0.25j, 0.4
    lam = c + r * RNG.uniform(0.1, 2.0, n) * np.exp(1j * RNG.uniform(0, 2 * np.pi, n))
    b = RNG.uniform(0.5, 1.5, n)
    A, B = W.diagonal_pencil(lam, b)
    Y = W.start_block(n, 5, 3)
    got = filters.simple_filter(A, B, c, r, k, Y)
    want = _compact(lam, c, r, k)[:, None] * Y
    assert _relerr(got, want) <= 1e-13


@pytest.mark.parametrize("n", [50, 201])
def test_simple_filter_balanced_toeplitz(n):
    wl = W.toeplitz_workload(n=n, w=4, count=6)
    S = _dst(n)
    lam = W.toeplitz_eigs(n, 0, 1, W.TOEPLITZ_C)
    Y = W.start_block(n, 4, 1)
    k = wl.p * wl.q
    got = filters.simple_filter(wl.A, wl.B, wl.c, wl.r, k, Y)
    want = S @ (_compact(lam, wl.c, wl.r, k)[:, None] * (S @ Y))
    assert _relerr(got, want) <= 1e-11


def _convdiff_eig_1d(n, h, D, v):
    """Eigen-decomposition of the 1-D upwind operator (sub a, diag d, super e)."""
    dd = D / (h * h)
    a = -dd - max(v, 0.0) / h          # coefficient of u_{i-1}
    e = -dd + min(v, 0.0) / h          # coefficient of u_{i+1}
    d = 2 * dd + abs(v) / h
    j = np.arange(1, n + 1)
    rho = np.sqrt(a / e)                        # x_k = rho^k sin(k j pi/(n+1))
    lam = d + 2 * (a / rho) * np.cos(j * np.pi / (n + 1))
    S = _dst(n)
    scale = rho ** (j - 1)                      # diagonal similarity
    X = scale[:, None] * S
    Xinv = S / scale[None, :]
    return lam, X, Xinv


def test_simple_filter_convdiff_identity_mass():
    n, D, vel, shift = 8, 1.0, (20.0, 10.0), 0.05j
    h = 1.0 / (n + 1)
    A, B = W.convdiff_pencil(n, D, vel, shift, mass=None)
    lx, Xx, Xix = _convdiff_eig_1d(n, h, D, vel[0])
    ly, Xy, Xiy = _convdiff_eig_1d(n, h, D, vel[1])
    lam = (ly[:, None] + lx[None, :]).ravel() + shift   # index iy*n + ix
    X = np.kron(Xy, Xx)
    Xi = np.kron(Xiy, Xix)
    # the decomposition is exact: A X = X diag(lam)
    assert np.linalg.norm(A @ X - X * lam[None, :]) <= 1e-11 * np.linalg.norm(A.toarray())
    c = np.median(lam.real) + 0.05j
    r = 0.5 * np.sort(np.abs(lam - c))[9:11].sum()
    Y = W.start_block(n * n, 3, 5)
    k = 16
    got = filters.simple_filter(A, B, c, r, k, Y)
    want = X @ (_compact(lam, c, r, k)[:, None] * (Xi @ Y))
    assert _relerr(got, want) <= 1e-10


@pytest.mark.parametrize("p,q", [(4, 4), (4, 8), (2, 3)])
def test_composite_equals_simple_rule(p, q):
    # Thm. Rcrm at matrix level: composite path == simple rule with pq poles
    n = 12
    A, B = W.convdiff_pencil(n, 1.0, (20.0, 10.0), 0.05j, (0.5, 1.5), seed=2)
    lam = np.linalg.eigvals(np.linalg.solve(B.toarray(), A.toarray()))
    c = np.sort(lam.real)[40] + 0.05j
    r = 0.5 * np.sort(np.abs(lam - c))[11:13].sum()
    Y = W.start_block(n * n, 6, 9)
    G = filters.InnerOperator(A, B, c, r, p)
    s, cw, extra = coeffs.outer_shifts(q)
    U, _, iters, conv = gmres.composite_filter_apply(G, Y, s, cw, extra, tol=1e-14,
                                                     max_iter=n * n)
    assert conv.all()
    want = filters.simple_filter(A, B, c, r, p * q, Y)
    assert _relerr(U, want) <= 1e-10


def test_inner_operator_counts_applications():
    # Table circuitbehavior accounting: G is applied to n_col vectors for
    # Ytilde, then once per Arnoldi step per column
    n = 10
    A, B = W.convdiff_pencil(n, 1.0, (20.0, 10.0), 0.05j, (0.5, 1.5), seed=4)
    G = filters.InnerOperator(A, B, 3000 + 0.05j, 800.0, 4)
    s, cw, extra = coeffs.outer_shifts(4)
    Y = W.start_block(n * n, 5, 1)
    _, _, iters, _ = gmres.composite_filter_apply(G, Y, s, cw, extra, tol=1e-12)
    assert G.applications == 5 + int(iters.sum())


def test_multishift_gmres_matches_dense_shifted_solves():
    # Each shifted system (G - s_j I) u = y solved densely (numpy LU) on a
    # small pencil; the multi-shift GMRES answers must agree.
    n = 9
    A, B = W.convdiff_pencil(n, 1.0, (20.0, 10.0), 0.05j, (0.5, 1.5), seed=6)
    Ad, Bd = A.toarray(), B.toarray()
    c, r, p = 900 + 0.05j, 300.0, 4
    poles, wts = coeffs.trapezoid_nodes(c, r, p)
    Gd = sum(wi * np.linalg.solve(pi * Bd - Ad, Bd) for pi, wi in zip(poles, wts))
    G = filters.InnerOperator(A, B, c, r, p)
    assert np.linalg.norm(G(np.eye(n * n)) - Gd) <= 1e-11 * np.linalg.norm(Gd)
    s, _, _ = coeffs.outer_shifts(8)
    Y = W.start_block(n * n, 3, 2)
    Us, iters, conv = gmres.multishift_gmres(G, Y, s, tol=1e-14, max_iter=n * n)
    for sj, Uj in zip(s, Us):
        want = np.linalg.solve(Gd - sj * np.eye(n * n), Y)
        assert _relerr(Uj, want) <= 1e-10


def test_paper_solve_count_identity_fixture():
    # Table circuitbehavior (App. A): composite triangular solves per subspace
    # iteration = k1 * (n_col + sum of per-column GMRES steps).  The printed
    # counts are divisible by k1 = 8 and leave a per-column step total no larger
    # than n_col * (max step count), the identity our counters follow.
    import json, os
    path = os.path.join(os.path.dirname(__file__), "golden", "circuit_solve_counts.json")
    data = json.load(open(path))
    for row in data["rows"]:
        for solves, nmax in zip(row["composite_solves"], row["composite_n_iter"]):
            assert solves % data["k1"] == 0
            steps = solves // data["k1"] - data["n_col"]
            assert 0 < steps <= data["n_col"] * nmax
        for solves in row["simple_solves"]:
            assert solves == data["k"] * data["n_col"]
