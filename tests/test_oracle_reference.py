"""Pins of the oracle's large-pencil references (oracle/reference.py) and of the
pole-subset form of the simple rule (oracle/filters.py), on the CPU."""
import numpy as np
import scipy.linalg as sl

from oracle import filters, reference
from paper_2310_18043_amd import workloads as W


def test_nearest_eigenvalues_match_dense_qz():
    # random-mass convection-diffusion pencil, N = 400: shift-invert Arnoldi vs dense QZ
    A, B = W.convdiff_pencil(20, mass=(0.5, 1.5), seed=2)
    sigma = 1500.0 + 0.05j
    got = reference.nearest_eigenvalues(A, B, sigma, 30)
    lam = sl.eigvals(A.toarray(), B.toarray())
    want = lam[np.argsort(np.abs(lam - sigma))][:30]
    # the 30 nearest as sets (the ordering of near-equal distances may differ)
    d = np.abs(got[:, None] - want[None, :]).min(axis=1)
    assert np.all(d <= 1e-9 * np.abs(want).max())


def test_nearest_eigenvalues_toeplitz_closed_form():
    wl = W.toeplitz_workload(n=400, w=16, count=10)
    got = reference.nearest_eigenvalues(wl.A, wl.B, wl.c, 10)
    exact = W.toeplitz_eigs(400, 0, 1, W.TOEPLITZ_C)
    want = exact[np.argsort(np.abs(exact - wl.c))][:10]
    assert np.abs(np.sort_complex(got) - np.sort_complex(want)).max() <= 1e-12


def test_disk_with_count_picks_the_widest_gap():
    lam = np.array([0.0, 1.0, 2.0, 2.1, 5.0, 5.05])
    c, r, s, ratio = reference.disk_with_count(lam, [0.0], [2, 3, 4])
    # distances 0, 1, 2, 2.1, 5, 5.05: count 4 has the ratio 5 / 2.1
    assert s == 4 and abs(r - 0.5 * (2.1 + 5.0)) < 1e-15 and abs(ratio - 5 / 2.1) < 1e-12


def test_simple_filter_terms_sum_to_the_simple_rule():
    A, B = W.convdiff_pencil(12, mass=(0.5, 1.5), seed=3)
    Y = W.start_block(A.shape[0], 3, seed=1)
    full = filters.simple_filter(A, B, 300 + 0.05j, 100.0, 8, Y)
    parts = [filters.simple_filter_terms(A, B, 300 + 0.05j, 100.0, 8, Y, idx)
             for idx in ([0, 1, 2], [3, 4], [5, 6, 7])]
    got = parts[0] + parts[1] + parts[2]
    assert np.linalg.norm(got - full) <= 1e-13 * np.linalg.norm(full)
    # a dropped term is visible
    assert np.linalg.norm(parts[0] + parts[1] - full) > 1e-3 * np.linalg.norm(full)
