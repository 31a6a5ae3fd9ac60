"""Textbook closed forms used to pin the oracle (independent of it).

Gaussian product theorem: prod_i exp(-a_i (x - C_i)^2) = K exp(-p (x - P)^2)
with p = sum a_i, P = sum a_i C_i / p, K = exp(-(sum a_i C_i^2 - p P^2)).
Polynomial prefactors are re-expanded around P and integrated with the
Gaussian moments  int u^k exp(-p u^2) du = Gamma((k+1)/2) / p^((k+1)/2)
(k even, zero for k odd).
"""

from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as P


def _norm(alpha, l):
    base = (2.0 * alpha / math.pi) ** 0.25
    return base if l == 0 else base * 2.0 * math.sqrt(alpha)


def _moment(k, p):
    if k % 2:
        return 0.0
    return math.gamma((k + 1) / 2.0) / p ** ((k + 1) / 2.0)


def _shift_poly(coeffs, d):
    """Coefficients in u of sum_k c_k (u + d)^k."""
    out = np.zeros(1)
    for k, c in enumerate(coeffs):
        out = P.polyadd(out, c * P.polypow([d, 1.0], k))
    return out


def gauss_integral(factors):
    """Integral over the real line of prod_f poly_f(x - B_f) exp(-a_f (x - C_f)^2).

    factors: list of (coeffs in (x - B), B, a, C)."""
    p = sum(f[2] for f in factors)
    Pc = sum(f[2] * f[3] for f in factors) / p
    K = math.exp(-(sum(f[2] * f[3] ** 2 for f in factors) - p * Pc * Pc))
    poly = np.ones(1)
    for coeffs, B, _, _ in factors:
        poly = P.polymul(poly, _shift_poly(coeffs, Pc - B))
    return K * sum(c * _moment(k, p) for k, c in enumerate(poly))


def _gto(alpha, l, A):
    """(coeffs in (x - A), A, alpha, A) of a normalised 1D primitive."""
    c = np.zeros(l + 1)
    c[l] = _norm(alpha, l)
    return (c, A, alpha, A)


def _dgto(alpha, l, A):
    """Derivative of the normalised primitive: N [l u^(l-1) - 2 alpha u^(l+1)]."""
    c = np.zeros(l + 2)
    if l >= 1:
        c[l - 1] += l
    c[l + 1] += -2.0 * alpha
    return (_norm(alpha, l) * c, A, alpha, A)


def overlap_1d(a1, l1, A1, a2, l2, A2):
    return gauss_integral([_gto(a1, l1, A1), _gto(a2, l2, A2)])


def dd_1d(a1, l1, A1, a2, l2, A2):
    """int g1' g2' dx (the 1D stiffness form; kinetic is half of it)."""
    return gauss_integral([_dgto(a1, l1, A1), _dgto(a2, l2, A2)])


def three_gauss_1d(a1, l1, A1, a2, l2, A2, t, C):
    """int g1 g2 exp(-t^2 (x - C)^2) dx."""
    return gauss_integral([_gto(a1, l1, A1), _gto(a2, l2, A2), (np.ones(1), C, t * t, C)])


def richardson(f_h, f_h2):
    """Eliminate the h^2 term from values at h and h/2."""
    return (4.0 * f_h2 - f_h) / 3.0


def richardson3(f_h, f_h2, f_h4):
    """Eliminate the h^2 and h^4 terms from values at h, h/2 and h/4."""
    r1 = richardson(f_h, f_h2)
    r2 = richardson(f_h2, f_h4)
    return (16.0 * r2 - r1) / 15.0
