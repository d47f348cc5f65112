"""The paper's circuit workload (App. B): the generator against the sizes and nonzero
counts the paper lists, and the oracle's Alg. composite on the n_x = 10 pencil against a
dense generalized eigen-decomposition."""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_2310_18043_amd import workloads as W


@pytest.mark.parametrize("nx,size,nnz", [(10, 1220, 7440), (100, 120020, 776040),
                                         (200, 480020, 3112040)])
def test_circuit_sizes_match_the_papers_table(nx, size, nnz):
    # Table "Matrix information" (App. A): size and nnz of G + C
    A, B = W.circuit_pencil(nx)
    assert A.shape == (size, size)
    assert (abs(A) + abs(B)).nnz == nnz


def test_circuit_structure():
    A, B = W.circuit_pencil(10)
    # B = diag(C_c, L): 1000 capacitances in [0.5, 1.5] 1e-3, 20 zero port entries,
    # 200 inductances in [0.5, 1.5] * 10 * 1e-4
    # (for n_x = 10 both ranges are [0.5e-3, 1.5e-3])
    b = B.diagonal().real
    assert np.sum(b == 0) == 20
    assert np.sum((b >= 0.5e-3) & (b <= 1.5e-3)) == 1200
    # the pencil is real, banded (natural ordering interleaved with the extra unknowns)
    assert np.all(A.data.imag == 0)
    coo = A.tocoo()
    assert np.max(np.abs(coo.row - coo.col)) <= 256


@pytest.mark.slow
def test_oracle_solve_region_on_circuit10_vs_dense():
    from oracle import solver
    wl = W.circuit_workload()
    Y0 = W.start_block(wl.n, wl.w, 0)
    ref = solver.solve_region(wl.A, wl.B, wl.c, wl.r, wl.p, wl.q, Y0, s_expected=wl.s_expected)
    w = sl.eigvals(wl.A.toarray(), wl.B.toarray())
    w = w[np.isfinite(w)]
    inside = w[np.abs(w - wl.c) < wl.r]
    assert ref.converged and len(ref.lam) == len(inside) == wl.s_expected
    d = np.abs(ref.lam[:, None] - inside[None, :]).min(axis=1)
    assert np.all(d <= 1e-10 * np.abs(ref.lam))
    assert ref.err.max() <= 1e-10
