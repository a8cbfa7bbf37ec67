"""Real 4-D hyperspherical harmonics (HH) in float64, from their definition.

TEST INFRASTRUCTURE: part of the FP64 oracle; the product never imports it.

Definition followed (Sec. 4.1, Eq. 2-3; Appendix A.1 and A.2):

    H_{nlm}(d, gamma) = A_{n,l} sin^l(gamma) C^{l+1}_{n-l}(cos gamma) Y_{lm}(d)
    A_{n,l}           = (2l)!! sqrt( 2 (n+1) (n-l)! / (pi (n+l+1)!) )

with 0 <= l <= n, -l <= m <= l, C^lambda_k the Gegenbauer polynomial and
Y_{lm} the orthonormal real spherical harmonic written in Cartesian form
(Appendix A.2): for m > 0 the cosine part Re((x + i y)^m), for m < 0 the
sine part Im((x + i y)^|m|), times the polynomial in z built from the
coefficients B_{k,lm}, and the prefactor sqrt((2l+1)/(4 pi)) sqrt((l-m)!/(l+m)!),
times sqrt(2) when m != 0.

Readings of the paper taken here (each is pinned by a test that does not
reuse these formulas):
  * the numerator of A_{n,l} is (n-l)!, not the printed (n-l+1)!; only the
    former makes the functions orthonormal on S^3;
  * the Gegenbauer upper index is l+1 (Eq. 2), not the n+l printed in the
    Cartesian form of Appendix A.2, and its degree is n-l;
  * the real spherical harmonic carries sqrt(2) for m != 0 (missing in the
    appendix's Cartesian prefactor) and no Condon-Shortley phase (none appears
    in B_{k,lm});
  * the 3-D factor is evaluated on the unit view direction d = (x, y, z) with
    the polar axis along z: the appendix's x2 is z, x3 is x and x4 is y;
  * the functions are taken in the order n = 0, 1, 2, ...; l = 0..n;
    m = -l..l and the first K of them are used (K = 5, 14, 30 are the
    complete sets n <= 1, 2, 3 of Table 3; K = 16 adds (3,0,0), (3,1,-1)).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np


def canonical_nlm(K: int) -> List[Tuple[int, int, int]]:
    """First K index triples (n, l, m) in the order n, then l, then m."""
    out: List[Tuple[int, int, int]] = []
    n = 0
    while len(out) < K:
        for l in range(n + 1):
            for m in range(-l, l + 1):
                if len(out) < K:
                    out.append((n, l, m))
        n += 1
    return out


def double_factorial(k: int) -> int:
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


def hh_norm(n: int, l: int) -> float:
    """A_{n,l} of Eq. 3 with the (n-l)! numerator."""
    return double_factorial(2 * l) * math.sqrt(
        2.0 * (n + 1) * math.factorial(n - l) / (math.pi * math.factorial(n + l + 1)))


def gegenbauer(k: int, lam: float, x):
    """C^lam_k(x) from its explicit finite sum
    sum_j (-1)^j Gamma(k-j+lam) / (Gamma(lam) j! (k-2j)!) (2x)^(k-2j)."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    for j in range(k // 2 + 1):
        coef = ((-1) ** j) * math.gamma(k - j + lam) / (
            math.gamma(lam) * math.factorial(j) * math.factorial(k - 2 * j))
        acc = acc + coef * (2.0 * x) ** (k - 2 * j)
    return acc


def legendre_poly_part(l: int, m: int, z):
    """sqrt((l-m)!/(l+m)!) * sum_k B_{k,lm} z^(l-2k-m)  (Appendix A.2), m >= 0,
    B_{k,lm} = (-1)^k 2^-l C(l,k) C(2l-2k,l) (l-2k)!/(l-2k-m)!."""
    z = np.asarray(z, dtype=np.float64)
    acc = np.zeros_like(z)
    for k in range((l - m) // 2 + 1):
        b = ((-1) ** k) * 2.0 ** (-l) * math.comb(l, k) * math.comb(2 * l - 2 * k, l) * (
            math.factorial(l - 2 * k) / math.factorial(l - 2 * k - m))
        acc = acc + b * z ** (l - 2 * k - m)
    return math.sqrt(math.factorial(l - m) / math.factorial(l + m)) * acc


def _re_im_power(m: int, x, y):
    """A_m = Re((x+iy)^m) and B_m = Im((x+iy)^m) from the binomial sums."""
    a = np.zeros_like(x)
    b = np.zeros_like(x)
    for p in range(m + 1):
        term = math.comb(m, p) * x ** p * y ** (m - p)
        a = a + term * math.cos((m - p) * math.pi / 2.0)
        b = b + term * math.sin((m - p) * math.pi / 2.0)
    return a, b


def real_sh(l: int, m: int, d):
    """Orthonormal real spherical harmonic Y_{lm} at unit directions d[..., 3]."""
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pref = math.sqrt((2 * l + 1) / (4.0 * math.pi))
    mm = abs(m)
    poly = legendre_poly_part(l, mm, z)
    if m == 0:
        return pref * poly
    a, b = _re_im_power(mm, x, y)
    return math.sqrt(2.0) * pref * poly * (a if m > 0 else b)


def hh_radial(n: int, l: int, gamma):
    """g_{nl}(gamma) = A_{n,l} sin^l(gamma) C^{l+1}_{n-l}(cos gamma)."""
    gamma = np.asarray(gamma, dtype=np.float64)
    return hh_norm(n, l) * np.sin(gamma) ** l * gegenbauer(n - l, l + 1.0, np.cos(gamma))


def hh_basis(K: int, d, gamma):
    """h[..., K]: the first K real HH at unit directions d[..., 3] and
    hyperangles gamma[...]. d must already be unit length."""
    d = np.asarray(d, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    cols = [hh_radial(n, l, gamma) * real_sh(l, m, d) for (n, l, m) in canonical_nlm(K)]
    return np.stack(cols, axis=-1)
