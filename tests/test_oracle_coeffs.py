"""Pins of the oracle's scalar coefficients against closed forms in the paper.

* Lemma compact (Sec. 4.3): R_{0,1,k}(z) = 1/(1+z^k); with centre and radius,
  R_{c,r,k}(z) = 1/(1 + ((z-c)/r)^k).  Worked examples k = 2, 4 (Sec. 4.3).
* Thm. Rcrm (Sec. 5): R_{c,r,pq}(z) = sum_j c'_j (R_{c,r,p}(z) - s_j)^{-1} R_{c,r,p}(z)
  (+ (1/q) R_{c,r,p} for odd q).
* Prop. poles (Sec. 5): R_{c,r,p}(p_i^{(pq)}) is one of the s_j.
* Corollary of Sec. 4.4: the separation of R_{0,a,k} over the annulus
  a < |z| < b is 2/((b/a)^k - 1).
* Derived facts: Re s_j = 1/2 and sum_j c'_j = 1/2 for even q (the filter is
  1/2 on the contour's pole images).
"""
import numpy as np
import pytest

from oracle import coeffs

RNG = np.random.default_rng(20231018)


def _compact(z, c, r, k):
    return 1.0 / (1.0 + ((z - c) / r) ** k)


def _sample_points(c, r, m=400):
    # points spread over |z - c| in (0, 3r), kept away from the contour
    rad = r * RNG.uniform(0.0, 3.0, m)
    rad = np.where(np.abs(rad - r) < 0.05 * r, rad + 0.1 * r, rad)
    ang = RNG.uniform(0, 2 * np.pi, m)
    return c + rad * np.exp(1j * ang)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("c,r", [(0.0, 1.0), (0.3 + 0.2j, 0.031623), (2525 + 0.05j, 661.5)])
def test_compact_form(k, c, r):
    z = _sample_points(c, r)
    got = coeffs.rational_filter(z, c, r, k)
    want = _compact(z, c, r, k)
    assert np.max(np.abs(got - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))


def test_worked_examples_k2_k4():
    # Sec. 4.3: R_{0,1,2}(z) = 1/(1+z^2) and R_{0,1,4}(z) = R_{0,1,2}(z^2)
    z = _sample_points(0.0, 1.0)
    assert np.allclose(coeffs.rational_filter(z, 0, 1, 2), 1 / (1 + z * z), rtol=0, atol=1e-14)
    assert np.allclose(coeffs.rational_filter(z, 0, 1, 4),
                       coeffs.rational_filter(z * z, 0, 1, 2), rtol=0, atol=1e-14)


def test_nodes_match_paper_values_k2():
    # Sec. 4.3 worked example: the two poles of R_{0,1,2} are e^{i pi/2}, e^{3 i pi/2}
    poles, w = coeffs.trapezoid_nodes(0.0, 1.0, 2)
    assert np.allclose(poles, [1j, -1j], atol=1e-15)
    assert np.allclose(w, [0.5j, -0.5j], atol=1e-15)


@pytest.mark.parametrize("p,q", [(4, 4), (4, 8), (8, 8), (2, 2), (4, 3), (2, 5), (3, 1)])
def test_composite_identity(p, q):
    c, r = 0.3 + 0.2j, 0.05
    z = _sample_points(c, r)
    got = coeffs.composite_filter(z, c, r, p, q)
    want = _compact(z, c, r, p * q)
    assert np.max(np.abs(got - want)) <= 1e-11


def test_paper_literal_outer_weights_give_negative_filter():
    # The statement of eq. Rcrm_ (c_i = -c'_i with (R - s_i)^{-1} R) sums to -R_{pq};
    # the oracle's sign reading is the one that reproduces +R_{pq}.
    c, r, p, q = 0.0, 1.0, 4, 8
    z = _sample_points(c, r)
    rp = coeffs.rational_filter(z, c, r, p)
    s, cw, _ = coeffs.outer_shifts(q)
    literal = sum(-cj * rp / (rp - sj) for sj, cj in zip(s, cw))
    assert np.max(np.abs(literal + _compact(z, c, r, p * q))) <= 1e-11


@pytest.mark.parametrize("p,q", [(4, 4), (4, 8), (8, 8)])
def test_pole_mapping(p, q):
    # Prop. poles: the inner filter maps every pole of the pq-rule onto an outer shift
    c, r = 1.0 + 2.0j, 3.0
    big, _ = coeffs.trapezoid_nodes(c, r, p * q)
    s, _, _ = coeffs.outer_shifts(q)
    img = coeffs.rational_filter(big, c, r, p)
    dist = np.min(np.abs(img[:, None] - s[None, :]), axis=1)
    assert dist.max() <= 1e-12


@pytest.mark.parametrize("q", [2, 4, 8, 16])
def test_shift_line_and_weight_sum(q):
    s, cw, extra = coeffs.outer_shifts(q)
    assert extra == 0.0 and len(s) == q
    assert np.allclose(s.real, 0.5, atol=1e-14)
    assert abs(cw.sum() - 0.5) <= 1e-14


@pytest.mark.parametrize("k", [2, 8, 16, 64])
def test_separation_corollary(k):
    # Corollary (Sec. 4.4) with a = 1, b = 1.1 (the setting of Sec. 6.1)
    a, b = 1.0, 1.1
    th = np.linspace(0, 2 * np.pi, 20001)
    # maximum modulus: extremes over I and O sit on |z| = a and |z| = b
    inner = np.abs(coeffs.rational_filter(a * np.exp(1j * th) * (1 - 1e-12), 0.0, a, k)).min()
    outer = np.abs(coeffs.rational_filter(b * np.exp(1j * th), 0.0, a, k)).max()
    want = 2.0 / ((b / a) ** k - 1.0)
    assert abs(outer / inner - want) <= 1e-6 * want


def test_mobius_inverts_inner_filter():
    # Sec. 5: M(R_{0,1,k1}(z)) = z^{k1}
    z = _sample_points(0.0, 1.0)
    for k1 in (2, 4, 8):
        got = coeffs.mobius(coeffs.rational_filter(z, 0.0, 1.0, k1))
        assert np.max(np.abs(got - z ** k1) / np.maximum(1, np.abs(z ** k1))) <= 1e-11
