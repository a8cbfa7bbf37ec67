"""Pins for the oracle's depth-aware alpha blending (Sec. 5.1, Alg. 1).

Reading: per pixel, sort the layers by depth (equal depth: the later layer is
in front, as Alg. 1's ``D_i <= D`` selects it), then premultiplied "over".
Pinned against Alg. 1 written literally for two layers, permutation
invariance, the exact render of a merged tree when the primitives are
separated in depth along every ray, and finite differences for the gradient.
"""
import math

import numpy as np

from oracle import core
from workloads import make_scene, orbit_camera


def alg1_literal(I, D, A):
    """Alg. 1 as printed, with straight colours I_i, on arrays over pixels."""
    Io, Do, Ao = I[0].copy(), D[0].copy(), A[0].copy()
    for i in range(1, I.shape[0]):
        fg = D[i] <= Do
        bg = ~fg
        new = Io.copy()
        new[fg] = A[i][fg, None] * I[i][fg] + (1 - A[i][fg, None]) * Ao[fg, None] * Io[fg]
        new[bg] = Ao[bg, None] * Io[bg] + (1 - Ao[bg, None]) * A[i][bg, None] * I[i][bg]
        Io = new
        Do = np.where(fg, D[i], Do)
        Ao = Ao + A[i] * (1 - Ao)
    return Io, Do, Ao


def test_two_layers_equal_literal_alg1():
    rng = np.random.default_rng(0)
    n = 500
    A = rng.uniform(0.01, 1, (2, n))
    I = rng.uniform(0, 1, (2, n, 3))
    D = rng.uniform(1, 5, (2, n))
    D[:, :50] = 2.0                      # ties: the later layer wins
    P = I * A[..., None]
    rgb, a, d = core.compose(P, A, D)
    Il, Dl, Al = alg1_literal(I, D, A)
    assert np.abs(rgb - Il).max() < 1e-14
    assert np.abs(a - Al).max() < 1e-14
    assert np.array_equal(d, Dl)


def test_tie_puts_later_layer_in_front():
    P = np.array([[[0.5, 0, 0]], [[0, 0.5, 0]], [[0, 0, 0.5]]])
    A = np.full((3, 1), 0.5)
    D = np.full((3, 1), 1.0)
    rgb, a, d = core.compose(P, A, D)
    assert np.allclose(rgb[0], [0.125, 0.25, 0.5])


def test_permutation_invariance():
    rng = np.random.default_rng(1)
    L, n = 5, 300
    P = rng.uniform(0, 0.5, (L, n, 3))
    A = rng.uniform(0, 1, (L, n))
    D = rng.uniform(0, 10, (L, n))
    D[2, :20] = np.inf
    ref = core.compose(P, A, D)
    perm = rng.permutation(L)
    out = core.compose(P[perm], A[perm], D[perm])
    for x, y in zip(ref, out):
        assert np.abs(x - y).max() < 1e-14


def test_depth_separated_primitives_equal_merged_render(oracle_lib):
    sc = make_scene(5, 4000, "random", seed=9, T=10)
    G = sc.G
    front = sc.leaf_ijk[:, 0] < G // 2
    cam = orbit_camera((G / 2, G / 2, G / 2), 3.0 * G, math.pi, 0.0, 48, 48, 30.0)  # on the -x side
    o, d = oracle_lib.pinhole_rays(48, 48, cam.intr(), cam.c2w)
    assert np.all(d[:, 0] > 0)
    args = lambda m: (5, sc.leaf_ijk[m], sc.hh[m], sc.wsig[m], sc.basis, sc.gamma, o, d, None, 4.0, 0.0)
    ra, rb = oracle_lib.render(*args(front)), oracle_lib.render(*args(~front))
    merged = oracle_lib.render(*args(np.ones_like(front)))
    rgb, a, dep = core.compose(np.stack([rb["rgb"], ra["rgb"]]), np.stack([rb["alpha"], ra["alpha"]]),
                               np.stack([rb["depth"], ra["depth"]]))
    assert merged["alpha"].max() > 0.5
    assert np.abs(rgb - merged["rgb"]).max() < 1e-12
    assert np.abs(a - merged["alpha"]).max() < 1e-12


def test_compose_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    L, n = 4, 40
    P = rng.uniform(0, 0.5, (L, n, 3))
    A = rng.uniform(0.05, 0.95, (L, n))
    D = rng.uniform(0, 10, (L, n))
    gP = rng.normal(size=(n, 3))
    gA = rng.normal(size=n)
    loss = lambda P_, A_: float((core.compose(P_, A_, D)[0] * gP).sum() + (core.compose(P_, A_, D)[1] * gA).sum())
    dP, dA = core.compose_grad(P, A, D, gP, gA)
    eps = 1e-6
    for (l, i, c) in [(0, 0, 0), (1, 3, 2), (3, 7, 1), (2, 11, 0)]:
        Pp = P.copy(); Pp[l, i, c] += eps
        Pm = P.copy(); Pm[l, i, c] -= eps
        assert abs((loss(Pp, A) - loss(Pm, A)) / (2 * eps) - dP[l, i, c]) < 1e-8
    for (l, i) in [(0, 0), (1, 5), (2, 9), (3, 13), (0, 21)]:
        Ap = A.copy(); Ap[l, i] += eps
        Am = A.copy(); Am[l, i] -= eps
        assert abs((loss(P, Ap) - loss(P, Am)) / (2 * eps) - dA[l, i]) < 1e-8
