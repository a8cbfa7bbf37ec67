"""Pins for the oracle's hyperspherical-harmonic basis (Sec. 4.1 Eq. 2-3, Appendix A.1-A.2).

Nothing here re-types the oracle's formulas: the basis is checked against
orthonormality on S^3 by quadrature, against scipy's Gegenbauer polynomials
and complex spherical harmonics, against the trigonometric closed form of the
l = 0 family, and against harmonicity of its homogeneous extension in R^4.
Two planted mistakes (the printed normalisation, the appendix's Gegenbauer
index) are shown to fail these pins.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_gegenbauer, roots_legendre, sph_harm_y

from oracle import hh as H


def s3_quadrature(ng=24, nt=24, nphi=48):
    xg, wg = roots_legendre(ng)
    gam = (xg + 1) * math.pi / 2
    wgam = wg * math.pi / 2 * np.sin(gam) ** 2
    ct, wt = roots_legendre(nt)
    phi = np.arange(nphi) * 2 * math.pi / nphi
    wphi = np.full(nphi, 2 * math.pi / nphi)
    G, CT, P = np.meshgrid(gam, ct, phi, indexing="ij")
    W = (wgam[:, None, None] * wt[None, :, None] * wphi[None, None, :]).reshape(-1)
    st = np.sqrt(1 - CT ** 2)
    d = np.stack([st * np.cos(P), st * np.sin(P), CT], -1).reshape(-1, 3)
    return d, G.reshape(-1), W


def gram(basis_fn, K):
    d, g, w = s3_quadrature()
    h = basis_fn(K, d, g)
    return (h * w[:, None]).T @ h


@pytest.mark.parametrize("K", [5, 14, 16, 30])
def test_gram_is_identity(K):
    assert np.abs(gram(H.hh_basis, K) - np.eye(K)).max() < 1e-12


def test_c_oracle_gram_and_agreement(oracle_lib):
    d, g, w = s3_quadrature()
    hc = oracle_lib.hh_basis_c(30, d, g)
    hn = H.hh_basis(30, d, g)
    assert np.abs(hc - hn).max() < 1e-12
    G = (hc * w[:, None]).T @ hc
    assert np.abs(G - np.eye(30)).max() < 1e-12


def test_canonical_order_counts():
    assert [len(H.canonical_nlm(k)) for k in (5, 14, 30)] == [5, 14, 30]
    full = H.canonical_nlm(30)
    assert {t for t in full if t[0] <= 1} == set(H.canonical_nlm(5))
    assert {t for t in full if t[0] <= 2} == set(H.canonical_nlm(14))
    assert H.canonical_nlm(16)[14:] == [(3, 0, 0), (3, 1, -1)]
    # 14 HH x 3 channels + 31 density + 31 hyperangle weights = the 104-dim leaf vector (Sec. 1)
    assert 14 * 3 + 31 + 31 == 104


def real_sh_scipy(l, m, d):
    """Real SH without Condon-Shortley phase from scipy's complex SH (which carries it)."""
    theta = np.arccos(np.clip(d[..., 2], -1, 1))
    phi = np.arctan2(d[..., 1], d[..., 0])
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    s = math.sqrt(2) * (-1) ** abs(m)
    return s * (np.real(y) if m > 0 else np.imag(y))


def test_against_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.uniform(0, math.pi, 200)
    h = H.hh_basis(30, d, g)
    for k, (n, l, m) in enumerate(H.canonical_nlm(30)):
        A = H.double_factorial(2 * l) * math.sqrt(2 * (n + 1) * math.factorial(n - l) /
                                                   (math.pi * math.factorial(n + l + 1)))
        ref = A * np.sin(g) ** l * eval_gegenbauer(n - l, l + 1, np.cos(g)) * real_sh_scipy(l, m, d)
        assert np.abs(h[:, k] - ref).max() < 1e-12, (n, l, m)


def test_closed_forms():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.uniform(0.01, math.pi - 0.01, 50)
    h = H.hh_basis(30, d, g)
    # H_000 = 1 / sqrt(|S^3|) = 1 / (pi sqrt 2)
    assert np.abs(h[:, 0] - 1 / (math.pi * math.sqrt(2))).max() < 1e-15
    # l = 0 family: A_{n,0} C^1_n(cos g) Y_00 with C^1_n = U_n = sin((n+1) g) / sin g
    for k, (n, l, m) in enumerate(H.canonical_nlm(30)):
        if l == 0:
            ref = math.sqrt(2 / math.pi) * np.sin((n + 1) * g) / np.sin(g) / math.sqrt(4 * math.pi)
            assert np.abs(h[:, k] - ref).max() < 1e-12
    # degree-1 real SH are the Cartesian components times sqrt(3/(4 pi)), ordered y, z, x
    c1 = math.sqrt(3 / (4 * math.pi)) * H.hh_radial(1, 1, g)
    assert np.abs(h[:, 2] - c1 * d[:, 1]).max() < 1e-14
    assert np.abs(h[:, 3] - c1 * d[:, 2]).max() < 1e-14
    assert np.abs(h[:, 4] - c1 * d[:, 0]).max() < 1e-14


def _hh_from_r4(fn_basis, x, K):
    """Homogeneous extension |x|^n H(x/|x|) of each basis function at points x [.,4]."""
    r = np.linalg.norm(x, axis=1)
    cg = x[:, 0] / r
    v = x[:, 1:]
    sv = np.linalg.norm(v, axis=1)
    g = np.arccos(np.clip(cg, -1, 1))
    d = np.stack([v[:, 1], v[:, 2], v[:, 0]], -1) / sv[:, None]   # (x3, x4, x2) -> (x, y, z)
    h = fn_basis(K, d, g)
    ns = np.array([n for (n, _, _) in H.canonical_nlm(K)])
    return h * r[:, None] ** ns[None, :]


def harmonic_residual(fn_basis, K=30):
    rng = np.random.default_rng(2)
    x0 = rng.normal(size=(20, 4))
    x0 /= np.linalg.norm(x0, axis=1, keepdims=True)
    e = 1e-3
    lap = -8 * _hh_from_r4(fn_basis, x0, K)
    for a in range(4):
        dx = np.zeros(4)
        dx[a] = e
        lap += _hh_from_r4(fn_basis, x0 + dx, K) + _hh_from_r4(fn_basis, x0 - dx, K)
    return np.abs(lap / e ** 2).max()


def test_homogeneous_extension_is_harmonic():
    # the degree-n HH are restrictions of harmonic polynomials on R^4
    assert harmonic_residual(H.hh_basis) < 1e-4


def test_planted_printed_normalisation_fails(monkeypatch):
    printed = lambda n, l: H.double_factorial(2 * l) * math.sqrt(
        2.0 * (n + 1) * math.factorial(n - l + 1) / (math.pi * math.factorial(n + l + 1)))
    monkeypatch.setattr(H, "hh_norm", printed)
    assert np.abs(gram(H.hh_basis, 14) - np.eye(14)).max() > 0.5


def test_planted_appendix_gegenbauer_index_fails(monkeypatch):
    def radial(n, l, gamma):
        gamma = np.asarray(gamma, np.float64)
        lam = max(n + l, 1)    # C^0 is degenerate; the appendix index only differs from n >= 1 on
        return H.hh_norm(n, l) * np.sin(gamma) ** l * H.gegenbauer(n - l, lam, np.cos(gamma))
    monkeypatch.setattr(H, "hh_radial", radial)
    assert harmonic_residual(H.hh_basis) > 1e-1
    assert np.abs(gram(H.hh_basis, 14) - np.eye(14)).max() > 0.5


def test_planted_condon_shortley_sign_fails(monkeypatch):
    orig = H.real_sh
    monkeypatch.setattr(H, "real_sh", lambda l, m, d: (-1) ** abs(m) * orig(l, m, d))
    rng = np.random.default_rng(3)
    d = rng.normal(size=(10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.uniform(0, math.pi, 10)
    h = H.hh_basis(4, d, g)
    c1 = math.sqrt(3 / (4 * math.pi)) * H.hh_radial(1, 1, g)
    assert np.abs(h[:, 2] - c1 * d[:, 1]).max() > 1e-3
