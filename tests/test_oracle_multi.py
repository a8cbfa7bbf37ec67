"""Pins of the exact multi-instance merge oracle: one instance is the single
render; instances disjoint in depth give Alg. 1's per-pixel "over"; a
duplicated voxel has twice the optical depth; two half-overlapping voxels give
the three-interval closed form; the instance order does not matter."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import core as OC
from oracle import multi as OM
from workloads import make_scene, random_rays, special_rays


def scene_ns(ijk, hh, wsig, basis, gamma, depth=3):
    return SimpleNamespace(depth=depth, leaf_ijk=np.asarray(ijk, np.int32), hh=np.asarray(hh, np.float32),
                           wsig=np.asarray(wsig, np.float32), basis=np.asarray(basis, np.float32),
                           gamma=np.asarray(gamma, np.float32))


def rot_z(th):
    return np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], np.float32)


def test_one_instance_is_the_single_render():
    sc = make_scene(4, 1500, "random", seed=41, T=8)
    inst = OC.Instance(rot_z(0.4), np.array([1.5, -2.0, 0.5], np.float32), 1.25, 2.5, 1)
    rng = np.random.default_rng(42)
    o1, d1 = random_rays(sc.G, 300, rng, inside_frac=0.2)
    o2, d2 = special_rays(sc.G)
    o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
    for t_stop in (0.0, 1e-2):
        a = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 3.0, t_stop, inst)
        b = OM.render_multi([sc], [inst], o, d, 3.0, t_stop)
        assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12
        assert np.abs(a["alpha"] - b["alpha"]).max() < 1e-12
        assert np.array_equal(a["nsamp"], b["nsamp"])
        fin = np.isfinite(a["depth"])
        assert np.array_equal(fin, np.isfinite(b["depth"]))
        assert np.abs(a["depth"][fin] - b["depth"][fin]).max() < 1e-9


def test_disjoint_in_depth_is_alg1_over():
    sc = make_scene(4, 1500, "random", seed=43, T=8)
    G = sc.G
    near = OC.Instance(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 0.0, 0)
    far = OC.Instance(np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 3.0 * G], np.float32), 1.0, 1.0, 0)
    rng = np.random.default_rng(44)
    o = np.stack([rng.uniform(0, G, 200), rng.uniform(0, G, 200), np.full(200, -2.0 * G)], 1).astype(np.float32)
    d = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (200, 1))
    d[:, :2] = rng.normal(0, 0.01, (200, 2))
    A = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 2.0, 0.0, near)
    B = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 2.0, 0.0, far)
    rgb, alpha, depth = OC.compose(np.stack([A["rgb"], B["rgb"]]), np.stack([A["alpha"], B["alpha"]]),
                                   np.stack([A["depth"], B["depth"]]))
    M = OM.render_multi([sc, sc], [far, near], o, d, 2.0, 0.0)
    assert (A["nsamp"] > 0).sum() > 50 and (B["nsamp"] > 0).sum() > 50
    assert np.abs(M["rgb"] - rgb).max() < 1e-12 and np.abs(M["alpha"] - alpha).max() < 1e-12


def voxel():
    ijk = [[1, 1, 1]]
    hh = [[[0.7], [-0.4], [1.3]]]
    wsig = [[0.9]]
    basis = [[1.0]]
    gamma = [1.0]
    sc = scene_ns(ijk, hh, wsig, basis, gamma)
    sig = math.log1p(math.exp(float(sc.wsig[0, 0])))           # the float32 values the oracle is given
    h0 = 1.0 / (math.pi * math.sqrt(2.0))
    c = np.array([1 / (1 + math.exp(-float(v) * h0)) for v in sc.hh[0, :, 0]])
    return sc, sig, c


def test_duplicate_voxel_doubles_optical_depth():
    sc, sig, c = voxel()
    I = OC.Instance(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 0.0, 0)
    o = np.array([[1.5, 1.5, -3.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    M = OM.render_multi([sc, sc], [I, I], o, d, 0.0, 0.0)
    a = 1 - math.exp(-2 * sig)
    assert abs(M["alpha"][0] - a) < 1e-14 and np.abs(M["rgb"][0] - a * c).max() < 1e-14
    assert M["nsamp"][0] == 1 and abs(M["depth"][0] - 4.5) < 1e-12


def test_half_overlapping_voxels_closed_form():
    sc, sig, c = voxel()
    sc2 = scene_ns([[1, 1, 1]], [[[-1.1], [0.3], [0.2]]], [[0.1]], [[1.0]], [1.0])
    sig2 = math.log1p(math.exp(float(sc2.wsig[0, 0])))
    h0 = 1.0 / (math.pi * math.sqrt(2.0))
    c2 = np.array([1 / (1 + math.exp(-float(v) * h0)) for v in sc2.hh[0, :, 0]])
    I = OC.Instance(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 0.0, 0)
    J = OC.Instance(np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 0.5], np.float32), 1.0, 0.0, 0)
    o = np.array([[1.5, 1.5, -3.0]], np.float32)
    d = np.array([[0.0, 0.0, 2.0]], np.float32)          # |d| = 2: u runs at half the world speed
    M = OM.render_multi([sc, sc2], [I, J], o, d, 0.0, 0.0)
    # u intervals (world z = -3 + 2u): voxel A on z in [1, 2) -> u in [2, 2.5); B on [1.5, 2.5) -> [2.25, 2.75)
    ka, kb = sig * 2.0, sig2 * 2.0                       # extinction per unit u (|d_l| = 2)
    T = 1.0
    col = np.zeros(3)
    wsum = dsum = 0.0
    for (a, b), ks, cc in [((2.0, 2.25), [ka], [c]), ((2.25, 2.5), [ka, kb], [c, c2]), ((2.5, 2.75), [kb], [c2])]:
        tau = sum(ks) * (b - a)
        cm = sum(k * x for k, x in zip(ks, cc)) / sum(ks)
        w = T * (1 - math.exp(-tau))
        col += w * cm
        wsum += w
        dsum += w * 0.5 * (a + b) * 2.0
        T *= math.exp(-tau)
    assert M["nsamp"][0] == 3
    assert np.abs(M["rgb"][0] - col).max() < 1e-14 and abs(M["alpha"][0] - wsum) < 1e-14
    assert abs(M["depth"][0] - dsum / wsum) < 1e-12


def test_instance_order_does_not_matter():
    sc = make_scene(4, 1500, "random", seed=45, T=8)
    A = OC.Instance(rot_z(0.3), np.array([1.0, 2.0, 0.0], np.float32), 1.0, 0.0, 0)
    B = OC.Instance(rot_z(-0.5), np.array([-2.0, 1.0, 1.0], np.float32), 0.8, 3.0, 1)
    rng = np.random.default_rng(46)
    o, d = random_rays(sc.G, 200, rng, inside_frac=0.3)
    x = OM.render_multi([sc, sc], [A, B], o, d, 1.0, 1e-3)
    y = OM.render_multi([sc, sc], [B, A], o, d, 1.0, 1e-3)
    assert (x["nsamp"] > 0).sum() > 30
    assert np.abs(x["rgb"] - y["rgb"]).max() < 1e-12 and np.array_equal(x["nsamp"], y["nsamp"])
