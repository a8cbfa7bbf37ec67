"""Pins of the appearance-editing oracle (Sec. 5.2): inactive edits change
nothing; an active edit on a single voxel gives the closed form with the target
colour and density; the terminating voxel along a row of leaves of known
density is the one where 1 - T first exceeds the threshold; painting keeps the
lowest ray index per leaf."""
import math

import numpy as np
import pytest

from oracle import core as OC
from oracle import editing as OE
from workloads import random_rays, special_rays

from test_oracle_render import tiny_scene


def test_inactive_edits_change_nothing():
    ijk, hh, wsig, basis, gamma = tiny_scene(3, seed=4)
    rng = np.random.default_rng(5)
    o, d = random_rays(8, 60, rng, inside_frac=0.3)
    a = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 2.0, 0.05)
    e = OE.empty_edits(ijk.shape[0])
    e[:, :3] = 0.5
    e[:, 4] = 3.0                                   # becomes active only from frame 3 on
    b = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 2.0, 0.05, edit=e)
    for k in ("rgb", "alpha", "depth", "nsamp"):
        assert np.array_equal(a[k], b[k]), k


def test_single_voxel_edit_closed_form():
    ijk = np.array([[1, 2, 3]], np.int32)
    hh = np.array([[[0.7], [-0.4], [1.3]]], np.float32)
    wsig = np.array([[0.9, -0.3]], np.float32)
    basis = np.array([[1.0, 2.0], [0.5, -1.0], [0.2, 0.1]], np.float32)
    gamma = np.array([0.4, 1.1, 2.0], np.float32)
    o, d = np.array([[1.5, 2.5, -4.0]], np.float32), np.array([[0.0, 0.0, 1.0]], np.float32)
    cd = np.array([0.2, 0.9, 0.35])
    e = OE.empty_edits(1)
    e[0, :3], e[0, 3], e[0, 4] = cd, 2.5, 1.0
    x = float(wsig[0, 0]) * 1.0 + float(wsig[0, 1]) * 2.0      # frame 0: basis row 0
    sig0 = math.log1p(math.exp(x))
    before = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 0.0, 0.0, edit=e)
    assert abs(before["alpha"][0] - (1 - math.exp(-sig0))) < 1e-14        # t = 0 < t_d: original
    after = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 1.0, 0.0, edit=e)
    a = 1 - math.exp(-2.5)
    assert abs(after["alpha"][0] - a) < 1e-14 and np.abs(after["rgb"][0] - a * cd).max() < 1e-14
    e[0, 3] = -1.0                                                        # keep the leaf's density
    keep = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 2.0, 0.0, edit=e)
    x2 = float(wsig[0, 0]) * float(basis[2, 0]) + float(wsig[0, 1]) * float(basis[2, 1])
    a2 = 1 - math.exp(-math.log1p(math.exp(x2)))
    assert abs(keep["alpha"][0] - a2) < 1e-14 and np.abs(keep["rgb"][0] - a2 * cd).max() < 1e-14


def test_terminating_voxel_along_a_row():
    # leaves (i, 1, 1), i = 0..7, of density softplus(x_i); a ray along +x; the input order
    # is shuffled so that the leaf index is not the position
    rng = np.random.default_rng(7)
    xs = np.array([-3.0, -1.0, 0.2, 1.5, 0.0, 2.5, -2.0, 1.0])
    perm = rng.permutation(8)
    ijk = np.array([[i, 1, 1] for i in perm], np.int32)
    wsig = np.array([[xs[i]] for i in perm], np.float32)
    hh = np.zeros((8, 3, 1), np.float32)
    basis = np.ones((1, 1), np.float32)
    gamma = np.array([1.0], np.float32)
    sig = np.log1p(np.exp(wsig[:, 0].astype(np.float64)))
    o = np.array([[-5.0, 1.5, 1.5]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    for thr in (0.5, 0.9, 0.99, 0.999):
        res = OC.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 0.0, 1.0 - thr)
        tau = 0.0
        want = -1
        for pos in range(8):
            q = int(np.nonzero(perm == pos)[0][0])
            tau += sig[q]
            if 1.0 - math.exp(-tau) > thr:
                want = q
                break
        assert res["last_leaf"][0] == want, (thr, res["last_leaf"][0], want)


def test_paint_lowest_ray_wins():
    e = OE.empty_edits(4)
    last = np.array([2, -1, 2, 0, 3, 0])
    col = np.arange(18, dtype=np.float64).reshape(6, 3)
    out = OE.paint(e, last, col, 1.5, 7.0)
    assert np.array_equal(out[2], [0, 1, 2, 1.5, 7.0])      # rays 0 and 2 end in leaf 2: ray 0
    assert np.array_equal(out[0], [9, 10, 11, 1.5, 7.0])     # rays 3 and 5 in leaf 0: ray 3
    assert np.array_equal(out[3], [12, 13, 14, 1.5, 7.0])
    assert np.isinf(out[1, 4]) and out[1, 3] == -1.0
