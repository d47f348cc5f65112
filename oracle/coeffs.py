"""Scalar coefficients of the trapezoidal and composite rational filters.

Test infrastructure (oracle); never imported by the product path.
"""
from __future__ import annotations

import numpy as np


def trapezoid_nodes(c: complex, r: float, k: int):
    """Poles and weights of the k-point trapezoidal rule on |z - c| = r.

    eq. pwtp (Sec. 2.2): theta_i = (2i-1) pi / k, p_i = c + r e^{i theta_i},
    w_i = r e^{i theta_i} / k, for i = 1..k.
    """
    i = np.arange(1, k + 1)
    theta = (2 * i - 1) * np.pi / k
    e = np.exp(1j * theta)
    return complex(c) + r * e, r * e / k


def roots_of_minus_one(k: int):
    """The k roots of z^k = -1, sigma_i = e^{i (2i-1) pi / k} (Lemma compact)."""
    i = np.arange(1, k + 1)
    return np.exp(1j * (2 * i - 1) * np.pi / k)


def rational_filter(z, c: complex, r: float, k: int):
    """R_{c,r,k}(z) = sum_i w_i / (p_i - z)  (eq. discretizedCI with eq. pwtp)."""
    poles, weights = trapezoid_nodes(c, r, k)
    z = np.asarray(z, dtype=np.complex128)
    out = np.zeros_like(z)
    for pi, wi in zip(poles, weights):
        out = out + wi / (pi - z)
    return out


def outer_shifts(q: int):
    """Outer shifts s_j and weights c'_j of the composite rule.

    Thm. Rcrm (Sec. 5) with sigma_j the roots of z^q = -1:
    s_j = 1 / (1 + sigma_j).  Weight with the sign that makes the sum equal
    +R_{c,r,pq} when paired with (R_p - s_j)^{-1} R_p (the proof's last line):
    c'_j = (1/q) sigma_j / (1 + sigma_j).

    For odd q the root sigma = -1 has no finite shift; it is dropped here and
    its contribution (1/q) R_p is returned as ``extra`` (eq. Rcrmodd).
    """
    sig = roots_of_minus_one(q)
    finite = np.abs(1.0 + sig) > 1e-12
    s = 1.0 / (1.0 + sig[finite])
    cw = (1.0 / q) * sig[finite] / (1.0 + sig[finite])
    extra = 0.0 if q % 2 == 0 else 1.0 / q
    return s, cw, extra


def mobius(z):
    """M(z) = (1 - z) / z  (eq. mobiustrans, Sec. 5)."""
    z = np.asarray(z, dtype=np.complex128)
    return (1.0 - z) / z


def composite_filter(z, c: complex, r: float, p: int, q: int):
    """Summation form sum_j c'_j (R_p(z) - s_j)^{-1} R_p(z) (+ odd term).

    Thm. Rcrm (Sec. 5), eqs. Rcrm and Rcrmodd, with R_p = R_{c,r,p}.
    """
    rp = rational_filter(z, c, r, p)
    s, cw, extra = outer_shifts(q)
    out = extra * rp
    for sj, cj in zip(s, cw):
        out = out + cj * rp / (rp - sj)
    return out
