"""Pins of the input builders: the closed-form spectra used by the batched-disk
cases against dense eigenvalue solves, and the disk tiling's counts."""
import numpy as np
import pytest

from paper_2310_18043_amd import workloads as W


@pytest.mark.parametrize("v", [(20.0, 10.0), (-7.0, 3.0), (0.0, -15.0)])
def test_convdiff_const_eigs_against_dense_eig(v):
    n = 9
    A, B = W.convdiff_pencil(n, 1.0, v, 0.05j, None, 0)
    ev = np.sort_complex(np.linalg.eigvals(A.toarray()))
    cf = np.sort_complex(W.convdiff_const_eigs(n, 1.0, v, 0.05j))
    assert np.max(np.abs(ev - cf)) <= 1e-12 * np.max(np.abs(cf))


def test_toeplitz_eigs_against_dense_eig():
    A, _ = W.toeplitz_pencil(40, 0.3, 1.0, W.TOEPLITZ_C, balanced=False)
    ev = np.sort_complex(np.linalg.eigvals(A.toarray()))
    cf = np.sort_complex(W.toeplitz_eigs(40, 0.3, 1.0, W.TOEPLITZ_C))
    assert np.max(np.abs(ev - cf)) <= 1e-10


def test_disk_batch_counts_and_adjacency():
    A, B, disks, lam = W.disk_batch(n=128, ndisks=16)
    assert A.shape == (16384, 16384)
    prev_right = None
    for d in disks:
        inside = np.abs(lam - d["c"]) < d["r"]
        assert inside.sum() == d["count"]
        assert d["w"] >= 1.25 * d["count"] and d["w"] & (d["w"] - 1) == 0
        left, right = d["c"].real - d["r"], d["c"].real + d["r"]
        if prev_right is not None:
            assert abs(left - prev_right) <= 1e-9 * right
        prev_right = right
        # no eigenvalue within 2% of the radius of the rim
        dist = np.abs(np.abs(lam - d["c"]) / d["r"] - 1.0)
        assert dist.min() > 0.02


@pytest.mark.parametrize("v", [(20.0, 10.0), (-7.0, 3.0)])
def test_convdiff_const_cond_against_dense_left_right_vectors(v):
    import scipy.linalg as sl
    n = 9
    A, _ = W.convdiff_pencil(n, 1.0, v, 0.05j, None, 0)
    lam, vl, vr = sl.eig(A.toarray(), left=True, right=True)
    kap = (np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0)
           / np.abs(np.sum(vl.conj() * vr, axis=0)))
    cf_lam, cf_kap = W.convdiff_const_cond(n, 1.0, v, 0.05j)
    assert np.allclose(np.sort_complex(cf_lam), np.sort_complex(W.convdiff_const_eigs(n, 1.0, v)))
    for i in range(len(lam)):
        j = np.argmin(np.abs(cf_lam - lam[i]))
        assert abs(cf_kap[j] - kap[i]) <= 1e-6 * kap[i]


def test_strip_disks_are_adjacent_and_hold_their_counts():
    # eigenvalues on a thin strip (|Im| <= 2) with unit density along Re: each disk is
    # centred on the real axis, starts at or after the previous disk's right edge, and
    # holds exactly its reported count (its rim between two eigenvalues)
    rng = np.random.default_rng(3)
    lam = np.sort(rng.uniform(0, 2000, 2000)) + 1j * rng.uniform(-2, 2, 2000)
    counts = [10, 40, 25, 100, 15]
    disks = W.strip_disks(lam, counts, start=0.0)
    left = 0.0
    for (c, r, s), want in zip(disks, counts):
        assert c.imag == 0.0 and abs(s - want) <= 3
        assert c.real - r >= left - 1e-9
        d = np.abs(lam - c)
        assert int(np.sum(d < r)) == s
        assert np.min(np.abs(d - r)) > 0.0          # no eigenvalue on the rim
        left = c.real + r


def test_read_disk_table_cycles_outer_nodes(tmp_path):
    p = tmp_path / "disks.txt"
    p.write_text("# header\n0 10.0 0.0 5.0 12 16\n1 30.0 0.0 7.5 20 32\n2 60.0 0.0 9.0 33 64\n"
                 "3 90.0 0.5 3.0 10 16\n")
    disks = W.read_disk_table(str(p))
    assert [d["q"] for d in disks] == [4, 8, 16, 4]
    assert disks[3]["c"] == complex(90.0, 0.5) and disks[1]["w"] == 32 and disks[2]["count"] == 33
