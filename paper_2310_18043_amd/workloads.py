"""Seeded synthetic pencils, disks and start blocks.

This module only builds inputs: sparse matrices, a disk (centre, radius) and
random start blocks.  It holds none of the eigensolver's arithmetic (no
filters, no factorizations, no Krylov steps) and imports neither the oracle nor
the GPU binding, so the same bytes feed both sides of every parity check.

Pencils
-------
* Tridiagonal Toeplitz pencil (B = I): diagonal ``a``, super-diagonal ``b``,
  sub-diagonal ``c``.  Its eigenvalues are a + 2 sqrt(bc) cos(k pi/(n+1)).
  The *balanced* variant replaces both off-diagonals by sqrt(bc) (a diagonal
  similarity of the literal matrix): same eigenvalues, normal matrix.
* Convection-diffusion pencil: unit square, homogeneous Dirichlet boundary,
  n x n interior grid, h = 1/(n+1), natural ordering with x fastest.
  A = D * (5-point -Laplacian) + first-order upwind discretisation of v . grad
  (backward difference where the local velocity component is positive,
  forward difference where it is negative) + ``shift`` on the diagonal.
  B is a diagonal lumped mass with entries drawn Uniform[lo, hi] (or I).

All randomness comes from NumPy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Workload:
    """A pencil (A, B), a disk D(c, r) and the solver's shape parameters."""
    name: str
    A: sp.csr_matrix          # complex128 CSR
    B: sp.csr_matrix          # complex128 CSR
    c: complex                # disk centre
    r: float                  # disk radius
    p: int                    # inner (factorized) trapezoidal nodes
    q: int                    # outer (multi-shift GMRES) nodes
    w: int                    # block width n_col
    s_expected: Optional[int] = None   # eigenvalues expected inside D
    seed: int = 0

    @property
    def n(self) -> int:
        return self.A.shape[0]


# --------------------------------------------------------------------------
# pencils
# --------------------------------------------------------------------------

def toeplitz_pencil(n: int, a: complex, b: complex, c: complex,
                    balanced: bool = True):
    """Tridiagonal Toeplitz A (diag a, super b, sub c) and B = I (CSR c128)."""
    if balanced:
        beta = np.sqrt(complex(b) * complex(c))
        sup, sub = beta, beta
    else:
        sup, sub = complex(b), complex(c)
    main = np.full(n, complex(a), dtype=np.complex128)
    A = sp.diags([np.full(n - 1, sub), main, np.full(n - 1, sup)],
                 [-1, 0, 1], shape=(n, n), format="csr", dtype=np.complex128)
    B = sp.identity(n, dtype=np.complex128, format="csr")
    A.sort_indices()
    return A, B


def convdiff_pencil(n: int, diffusion: float = 1.0, velocity=(20.0, 10.0),
                    shift: complex = 0.05j, mass=(0.5, 1.5), seed: int = 0,
                    vfield: Optional[np.ndarray] = None):
    """Upwinded 5-point convection-diffusion pencil on an n x n grid.

    ``velocity`` is a constant (vx, vy); ``vfield`` (shape (2, n, n), indexed
    [component, iy, ix]) overrides it with a per-cell field.  ``mass`` is the
    Uniform range of the diagonal B, or None for B = I.  The mass draw uses
    ``seed``; a per-cell field is drawn by the caller.
    """
    h = 1.0 / (n + 1)
    N = n * n
    if vfield is None:
        vx = np.full((n, n), float(velocity[0]))
        vy = np.full((n, n), float(velocity[1]))
    else:
        vx = np.asarray(vfield[0], dtype=np.float64)
        vy = np.asarray(vfield[1], dtype=np.float64)
    dd = diffusion / (h * h)
    rows, cols, vals = [], [], []
    idx = np.arange(N).reshape(n, n)          # idx[iy, ix], x fastest
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    # diagonal: diffusion + upwind self terms + complex shift
    diag = 4.0 * dd + np.abs(vx) / h + np.abs(vy) / h + 0.0j
    diag = diag + shift
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())

    def couple(mask, di, dj, val):
        tgt = idx[(iy + di)[mask], (ix + dj)[mask]]
        rows.append(idx[mask]); cols.append(tgt); vals.append(val[mask] + 0.0j)

    # west neighbour (ix-1): diffusion -dd, upwind -vx/h when vx > 0
    m = ix > 0
    couple(m, 0, -1, -dd - np.where(vx > 0, vx, 0.0) / h)
    # east neighbour (ix+1): diffusion -dd, upwind +vx/h when vx < 0
    m = ix < n - 1
    couple(m, 0, 1, -dd + np.where(vx < 0, vx, 0.0) / h)
    # south neighbour (iy-1)
    m = iy > 0
    couple(m, -1, 0, -dd - np.where(vy > 0, vy, 0.0) / h)
    # north neighbour (iy+1)
    m = iy < n - 1
    couple(m, 1, 0, -dd + np.where(vy < 0, vy, 0.0) / h)

    A = sp.csr_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N), dtype=np.complex128)
    A.sum_duplicates(); A.sort_indices()
    if mass is None:
        B = sp.identity(N, dtype=np.complex128, format="csr")
    else:
        rng = np.random.Generator(np.random.PCG64(seed))
        bdiag = rng.uniform(mass[0], mass[1], size=N)
        B = sp.diags(bdiag.astype(np.complex128), 0, format="csr")
    B.sort_indices()
    return A, B


def random_vfield(n: int, vmax: float, seed: int) -> np.ndarray:
    """Per-cell convection field, Uniform[-vmax, vmax]^2, shape (2, n, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-vmax, vmax, size=(2, n, n))


def diagonal_pencil(lam: np.ndarray, bdiag: Optional[np.ndarray] = None):
    """A = diag(lam * b), B = diag(b): eigenvalues exactly ``lam``."""
    lam = np.asarray(lam, dtype=np.complex128)
    b = np.ones_like(lam) if bdiag is None else np.asarray(bdiag, np.complex128)
    A = sp.diags(lam * b, 0, format="csr", dtype=np.complex128)
    B = sp.diags(b, 0, format="csr", dtype=np.complex128)
    return A, B


def start_block(n: int, w: int, seed: int = 0) -> np.ndarray:
    """(randn + i randn)/sqrt(2), n x w, Fortran (column-major) order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((w, n))
    im = rng.standard_normal((w, n))
    Y = ((re + 1j * im) / np.sqrt(2.0)).T
    return np.asfortranarray(Y)


# --------------------------------------------------------------------------
# disks
# --------------------------------------------------------------------------

def midgap_radius(eigs: np.ndarray, c: complex, count: int) -> float:
    """Radius halfway between the count-th and (count+1)-th distance from c."""
    d = np.sort(np.abs(np.asarray(eigs) - c))
    return 0.5 * (d[count - 1] + d[count])


def toeplitz_eigs(n: int, a: complex, b: complex, c: complex) -> np.ndarray:
    """Closed-form eigenvalues a + 2 sqrt(bc) cos(k pi/(n+1)), k = 1..n."""
    k = np.arange(1, n + 1)
    return complex(a) + 2.0 * np.sqrt(complex(b) * complex(c)) * np.cos(k * np.pi / (n + 1))


def convdiff_const_eigs(n: int, diffusion: float = 1.0, velocity=(20.0, 10.0),
                        shift: complex = 0.05j) -> np.ndarray:
    """Closed-form eigenvalues of ``convdiff_pencil`` with constant velocity and B = I.

    A is then the Kronecker sum I (x) T_x + T_y (x) I of two tridiagonal Toeplitz
    matrices plus ``shift``; T_x has diagonal 2d + |v_x|/h and off-diagonals whose
    product is d (d + |v_x|/h), d = D/h^2 (the upwind side carries the |v_x|/h), so
    its eigenvalues follow the tridiagonal Toeplitz formula and those of A are all
    sums lambda_x(j) + lambda_y(k) + shift.  Returned sorted by real part."""
    h = 1.0 / (n + 1)
    d = diffusion / (h * h)

    def axis(v):
        u = abs(float(v)) / h
        return toeplitz_eigs(n, 2.0 * d + u, -d, -(d + u))

    lam = (axis(velocity[0])[:, None] + axis(velocity[1])[None, :]).ravel() + shift
    return lam[np.argsort(lam.real, kind="stable")]


def convdiff_const_cond(n: int, diffusion: float = 1.0, velocity=(20.0, 10.0),
                        shift: complex = 0.05j):
    """Eigenvalues (as ``convdiff_const_eigs``) and their condition numbers
    kappa = ||x|| ||y|| / |y^H x| for the same pencil.

    A tridiagonal Toeplitz matrix with off-diagonals sup, sub has right eigenvectors
    x_k = rho^k sin(k j pi/(n+1)) and left ones y_k = rho^-k sin(k j pi/(n+1)),
    rho = sqrt(sub/sup); for the Kronecker sum both factor as Kronecker products, so
    kappa is the product of the two axes' values.  A first-order bound on the error of
    a computed eigenvalue is kappa times the residual norm of its unit vector."""
    h = 1.0 / (n + 1)
    d = diffusion / (h * h)
    k = np.arange(1, n + 1)

    def axis(v):
        u = abs(float(v)) / h
        lam = toeplitz_eigs(n, 2.0 * d + u, -d, -(d + u))
        rho = np.sqrt((d + u) / d)
        S = np.sin(np.outer(k, k) * np.pi / (n + 1))        # S[k, j]
        # rho^k overflows nowhere for the grids used here (rho^n < 1e30)
        xr = np.linalg.norm(S * rho ** k[:, None], axis=0)
        yl = np.linalg.norm(S / rho ** k[:, None], axis=0)
        return lam, xr * yl / np.abs(np.sum(S * S, axis=0))

    lx, kx = axis(velocity[0])
    ly, ky = axis(velocity[1])
    lam = (lx[:, None] + ly[None, :]).ravel() + shift
    kap = (kx[:, None] * ky[None, :]).ravel()
    o = np.argsort(lam.real, kind="stable")
    return lam[o], kap[o]


def tile_disks(lam: np.ndarray, counts, start: int = 0, slack: int = 3):
    """Disks covering consecutive runs of eigenvalues lying on one horizontal line.

    ``lam`` sorted by real part, all with the same imaginary part.  Disk d takes
    about counts[d] eigenvalues following the previous disk's run: the run length is
    chosen within +-slack of the request to maximise the smaller of the two
    relative gaps at its ends, the disk's edges sit in the middle of those gaps.
    Returns a list of (c, r, count)."""
    x = np.real(lam)
    y = float(np.mean(np.imag(lam)))
    out = []
    i0 = start
    for want in counts:
        best = None
        for s in range(max(1, want - slack), want + slack + 1):
            if i0 + s >= len(x) or i0 + s - 1 < 0:
                continue
            lo = x[i0 - 1] if i0 > 0 else x[i0] - (x[i0 + 1] - x[i0])
            left = 0.5 * (lo + x[i0])
            right = 0.5 * (x[i0 + s - 1] + x[i0 + s])
            r = 0.5 * (right - left)
            gap = min(x[i0] - left, x[i0 + s] - right, right - x[i0 + s - 1]) / r
            if best is None or gap > best[0]:
                best = (gap, s, 0.5 * (left + right), r)
        _, s, cx, r = best
        out.append((complex(cx, y), float(r), int(s)))
        i0 += s
    return out


def strip_disks(lam: np.ndarray, counts, start: float, slack: int = 3, density_guess=None):
    """Adjacent disks centred on the real axis along a thin horizontal strip of
    eigenvalues (|Im| small against the radii), left to right from ``start``.

    Disk d is centred at L_d + r with L_d the previous disk's right edge (``start`` for
    the first): for every candidate count s within +-slack of counts[d] the radius is
    the one centred between the s-th and (s+1)-th nearest eigenvalues of a centre
    placed for about counts[d] eigenvalues (density from ``lam`` or ``density_guess``),
    and the candidate with the largest ratio of those two distances is kept.  ``lam``
    must hold every eigenvalue of the region the disks reach.  Returns a list of
    (c, r, count)."""
    lam = np.asarray(lam)
    x = np.sort(lam.real)
    dens = density_guess or (len(x) - 1) / (x[-1] - x[0])
    out = []
    left = float(start)
    for want in counts:
        half = 0.5 * want / dens
        best = None
        for shift in np.linspace(-0.3, 0.3, 13):
            cx = left + half * (1.0 + shift)
            d = np.sort(np.abs(lam - cx))
            for s in range(max(1, want - slack), want + slack + 1):
                r = 0.5 * (d[s - 1] + d[s])
                if cx - r < left - 1e-9 * abs(left):
                    continue                      # would reach back into the previous disk
                ratio = d[s] / d[s - 1]
                if best is None or ratio > best[3]:
                    best = (complex(cx, 0.0), float(r), int(s), float(ratio))
        if best is None:
            raise ValueError("no disk fits after %g" % left)
        out.append(best[:3])
        left = best[0].real + best[1]
    return out


def disk_batch(n: int = 128, ndisks: int = 16, lo: int = 12, hi: int = 48,
               seed: int = 0, velocity=(20.0, 10.0)):
    """Several adjacent disks at the low-|lambda| end of the constant-velocity
    convection-diffusion pencil with B = I (closed-form spectrum).

    Requested counts are log-uniform over [lo, hi] (PCG64, ``seed``); each disk's
    block width is the smallest power of two >= 1.25 x its count.  Returns
    (A, B, disks, exact_eigs) with disks a list of dicts c, r, w, count."""
    A, B = convdiff_pencil(n, 1.0, velocity, 0.05j, None, seed)
    lam = convdiff_const_eigs(n, 1.0, velocity, 0.05j)
    rng = np.random.Generator(np.random.PCG64(seed))
    want = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=ndisks))).astype(int)
    disks = []
    for c, r, s in tile_disks(lam, want):
        w = 16
        while w < 1.25 * s:
            w *= 2
        disks.append({"c": c, "r": r, "w": w, "count": s})
    return A, B, disks, lam


# --------------------------------------------------------------------------
# named workloads (shapes of the paper's experiments; sizes as in the
# composite-rule benchmark definitions)
# --------------------------------------------------------------------------

TOEPLITZ_C = 0.5 * np.exp(1j * np.pi / 3)

# Disk for the 128 x 128 convection-diffusion pencil (D = 1, v = (20, 10),
# +0.05i on the diagonal, B = diag U[0.5, 1.5] with seed 0).  Recipe: the 300
# eigenvalues of B^{-1}A nearest 2500 + 0.065i (ARPACK shift-invert); centres
# on the real line (imaginary part 0.0494, the strip's middle) scanned in steps
# of 5 over [1800, 3200); kept the centre whose 100th/101st distance ratio is
# largest; radius halfway between the 100th and 101st distances.
CONVDIFF128_DISK = (2525.0 + 0.0494j, 661.5612524628755, 100)

# Disk for the 128 x 128 pencil with a per-cell velocity field v ~ U[-20, 20]^2
# (random_vfield seed 5), D = 1, +0.05i, B = diag U[0.5, 1.5] (seed 0).  Recipe: the
# 200 eigenvalues of B^{-1}A nearest 2000 (ARPACK shift-invert, all within 1335 of
# 2000); centres on Im = 0.0495 scanned in steps of 2 over [1500, 2500) with counts
# 46..54 and the disk kept inside 0.9 x that range; kept the centre and count with
# the largest ratio of the (count+1)-th to the count-th distance (1.13); radius
# halfway between the two.
RANDOMV128_DISK = (1564.0 + 0.0495j, 350.8144063398522, 52)

# Disk for the 256 x 256 pencil with a per-cell velocity field v ~ U[-30, 30]^2
# (random_vfield seed 3), D = 1, +0.05i, B = diag U[0.5, 1.5] (seed 0).  Recipe
# (tests/golden/make_convdiff256.py): the 400 eigenvalues of B^{-1}A nearest 2000
# (ARPACK shift-invert, oracle.reference.nearest_eigenvalues; Re 20..5426, Im +-10.5);
# centres on the grid Re 1200..2795 step 5, Im -6..6 step 1, counts 185..215, keeping
# the disk (inside the computed set with 20% margin) with the largest ratio of the
# (count+1)-th to the count-th distance (1.045); radius halfway between the two.
CONVDIFF256_DISK = (2605.0 + 0.0j, 1255.9810842394086, 187)

_DISKS = {
    (128, (20.0, 10.0), 0, (0.5, 1.5)): CONVDIFF128_DISK,
}


def toeplitz_workload(n: int = 2000, balanced: bool = True, w: int = 32,
                      p: int = 4, q: int = 4, count: int = 20,
                      c: complex = 0.3 + 0.2j, seed: int = 0) -> Workload:
    A, B = toeplitz_pencil(n, 0.0, 1.0, TOEPLITZ_C, balanced=balanced)
    lam = toeplitz_eigs(n, 0.0, 1.0, TOEPLITZ_C)
    r = midgap_radius(lam, c, count)
    return Workload(f"toeplitz{'_bal' if balanced else '_lit'}_n{n}", A, B,
                    complex(c), float(r), p, q, w, count, seed)


def convdiff_workload(n: int = 128, w: int = 128, p: int = 4, q: int = 8,
                      seed: int = 0, velocity=(20.0, 10.0),
                      disk: Optional[tuple] = None,
                      mass=(0.5, 1.5)) -> Workload:
    A, B = convdiff_pencil(n, 1.0, velocity, 0.05j, mass, seed)
    if disk is None:
        disk = _DISKS.get((n, tuple(velocity), seed, mass))
    if disk is None:
        raise KeyError("no stored disk for this convection-diffusion pencil; "
                       "pass disk=(c, r, count)")
    c, r, count = disk
    return Workload(f"convdiff{n}", A, B, complex(c), float(r), p, q, w,
                    count, seed)


def random_velocity_workload(n: int = 128, w: int = 64, p: int = 4, q: int = 8,
                             vseed: int = 5, vmax: float = 20.0,
                             disk: Optional[tuple] = None) -> Workload:
    """Convection-diffusion pencil with a per-cell velocity field U[-vmax, vmax]^2
    (seed ``vseed``) and B = diag U[0.5, 1.5] (seed 0): the differentiation-form
    workload (gradients of eigenvalues with respect to the field)."""
    v = random_vfield(n, vmax, vseed)
    A, B = convdiff_pencil(n, 1.0, vfield=v, shift=0.05j, mass=(0.5, 1.5), seed=0)
    if disk is None:
        if (n, vseed, vmax) != (128, 5, 20.0):
            raise KeyError("no stored disk for this pencil; pass disk=(c, r, count)")
        disk = RANDOMV128_DISK
    c, r, count = disk
    wl = Workload(f"convdiff{n}_randv{vseed}", A, B, complex(c), float(r), p, q, w, count, 0)
    wl.vfield = v
    return wl


def convdiff256_workload(w: int = 256, p: int = 8, q: int = 8, vseed: int = 3,
                         vmax: float = 30.0) -> Workload:
    """The precision-form workload: 256 x 256 convection-diffusion pencil (N = 65536,
    bandwidth 256) with a per-cell velocity field U[-30, 30]^2 (seed 3), B = diag
    U[0.5, 1.5] (seed 0), +0.05i on the diagonal; disk with 187 eigenvalues
    (CONVDIFF256_DISK); p = q = 8, w = 256."""
    v = random_vfield(256, vmax, vseed)
    A, B = convdiff_pencil(256, 1.0, vfield=v, shift=0.05j, mass=(0.5, 1.5), seed=0)
    c, r, count = CONVDIFF256_DISK
    wl = Workload("convdiff256_randv3", A, B, complex(c), float(r), p, q, w, count, 0)
    wl.vfield = v
    return wl


def read_disk_table(path: str):
    """Disks of a batched workload from a text table (disk, Re c, Im c, r, count, w),
    as written by tests/golden/make_convdiff256_batch.py.  Outer node counts cycle
    through 4, 8, 16.  Returns a list of dicts c, r, count, w, q."""
    disks = []
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        d, cr, ci, r, count, w = line.split()
        disks.append({"c": complex(float(cr), float(ci)), "r": float(r), "count": int(count),
                      "w": int(w), "q": (4, 8, 16)[int(d) % 3]})
    return disks


# --------------------------------------------------------------------------
# the paper's circuit pencil (App. B, construction of the matrix)
# --------------------------------------------------------------------------

def _weighted_laplacian_1d(n: int):
    """(n / 100) tridiag(-1, 2, -1) with 1 in both corners (App. B)."""
    d = np.full(n, 2.0)
    d[0] = d[-1] = 1.0
    return (n / 100.0) * sp.diags([-np.ones(n - 1), d, -np.ones(n - 1)], [-1, 0, 1])


def circuit_pencil(nx: int, seed: int = 0, layers: int = 10):
    """Power-grid pencil of App. B on an nx x nx x 10 grid, as (A, B) = (-G, C).

    G = [[G11, G12], [-G12^T, 0]], C = diag(C_c, L):
      G11 = L_nx (x) I_nx (x) I_10 + I_nx (x) L_nx (x) I_10 + (1/10) I (x) I (x) L_10;
      G12: 20 input-port columns with a +1 at their node -- 10 ports spread along the
           edge (i, 1, 1) and 10 along (i, nx, 10) (all nodes of each edge when nx = 10) --
           and 2 nx^2 inductor columns, each joining a randomly picked interior node of a
           layer to a random one of its four neighbours on that layer (+1, -1);
      C_c = diag U[0.5, 1.5] 1e-3 (grounded capacitors), L = diag(0 (ports),
           U[0.5, 1.5] nx 1e-4 (inductances)).
    All draws from PCG64(seed) in that order: inductor nodes (without replacement),
    directions, capacitances, inductances.  For nx = 10 this gives the size (1220) and
    nonzero count of G + C (7440) the paper lists.

    The eigenvalue problem is taken as -G x = lambda C x (the circuit's poles, in the left
    half plane, where the paper's target regions lie).  Unknowns are ordered node by node,
    each port current right after its node and each inductor current after the node
    midway between its two nodes, so the pencil stays banded (bandwidth about 1.2 x 10 nx,
    128 for nx = 10).  Returns (A, B) as complex128 CSR."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nl = layers
    eye = lambda n: sp.identity(n)
    G11 = (sp.kron(sp.kron(_weighted_laplacian_1d(nx), eye(nx)), eye(nl))
           + sp.kron(sp.kron(eye(nx), _weighted_laplacian_1d(nx)), eye(nl))
           + 0.1 * sp.kron(sp.kron(eye(nx), eye(nx)), _weighted_laplacian_1d(nl)))
    nn = nx * nx * nl

    def node(i, j, l):
        return (i * nx + j) * nl + l

    extra = []                                    # (first node, rows, values)
    edge = np.unique(np.rint(np.linspace(0, nx - 1, 10)).astype(int))
    for i in edge:
        extra.append((node(i, 0, 0), [node(i, 0, 0)], [1.0]))
    for i in edge:
        extra.append((node(i, nx - 1, nl - 1), [node(i, nx - 1, nl - 1)], [1.0]))
    nports = len(extra)
    interior = [(i, j, l) for i in range(1, nx - 1) for j in range(1, nx - 1) for l in range(nl)]
    pick = rng.choice(len(interior), size=2 * nx * nx, replace=False)
    dirs = rng.integers(0, 4, size=len(pick))
    steps = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    for t, dsel in zip(pick, dirs):
        i, j, l = interior[t]
        di, dj = steps[dsel]
        a, b = node(i, j, l), node(i + di, j + dj, l)
        extra.append(((a + b) // 2, [a, b], [1.0, -1.0]))
    m = len(extra)
    cap = rng.uniform(0.5, 1.5, nn) * 1e-3
    ind = rng.uniform(0.5, 1.5, m - nports) * nx * 1e-4
    rows, cols, vals = [], [], []
    for k, (_, rr, vv) in enumerate(extra):
        rows += rr
        cols += [k] * len(rr)
        vals += vv
    G12 = sp.csr_matrix((vals, (rows, cols)), shape=(nn, m))
    G = sp.bmat([[G11, G12], [-G12.T, None]]).tocsr()
    C = sp.diags(np.concatenate([cap, np.zeros(nports), ind])).tocsr()
    # ordering: node k, then the extra unknowns placed at node k
    first = np.array([e[0] for e in extra])
    key = np.concatenate([np.arange(nn) * 2.0, first * 2.0 + 1.0])
    order = np.argsort(key, kind="stable")
    A = (-G)[order][:, order].astype(np.complex128).tocsr()
    B = C[order][:, order].astype(np.complex128).tocsr()
    A.sort_indices()
    B.sort_indices()
    return A, B


# Disk for circuit_pencil(10, seed 0): centre of the paper's n_x = 10 region,
# -200 + 1000i; of the dense eigenvalues of (-G, C), the counts 16..26 nearest the
# centre were scanned and 17 kept, whose 18th/17th distance ratio (1.13) is the
# largest near the paper's 20; radius halfway between the 17th and 18th distances.
CIRCUIT10_DISK = (-200.0 + 1000.0j, 71.3035740717, 17)


def circuit_workload(nx: int = 10, w: int = 24, p: int = 8, q: int = 8, seed: int = 0,
                     disk: Optional[tuple] = None) -> Workload:
    """The paper's circuit pencil (App. B) with the solver shape of its experiments
    (k1 = k2 = 8, n_col = 24)."""
    A, B = circuit_pencil(nx, seed)
    if disk is None:
        if (nx, seed) != (10, 0):
            raise KeyError("no stored disk for this circuit pencil; pass disk=(c, r, count)")
        disk = CIRCUIT10_DISK
    c, r, count = disk
    return Workload(f"circuit{nx}", A, B, complex(c), float(r), p, q, w, count, seed)
