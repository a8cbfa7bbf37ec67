"""Pins of the lighting oracle (Sec. 5.2 "Spotlight Lighting"): the Gaussian
low-pass against scipy, projection and sampling against hand-built cases,
shading against closed forms (ground hit point, inverse-square falloff,
premultiplied over, occlusion by the ground)."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import lighting as OL
from workloads import look_at


@pytest.mark.parametrize("sigma", [0.6, 1.0, 2.5, 4.0])
def test_blur_matches_scipy_gaussian_filter(sigma):
    rng = np.random.default_rng(int(sigma * 10))
    img = rng.random((37, 53))
    ref = ndimage.gaussian_filter(img, sigma, mode="nearest", truncate=3.0)
    assert np.abs(OL.blur(img, sigma) - ref).max() < 1e-12


def test_blur_invariants():
    w = OL.gaussian_weights(2.0)
    assert len(w) == 2 * 6 + 1 and abs(w.sum() - 1.0) < 1e-15 and np.allclose(w, w[::-1])
    const = np.full((20, 30), 0.37)
    assert np.abs(OL.blur(const, 2.0) - 0.37).max() < 1e-15
    imp = np.zeros((41, 41))
    imp[20, 20] = 1.0
    out = OL.blur(imp, 2.0)
    assert abs(out.sum() - 1.0) < 1e-12                       # interior impulse: mass kept
    assert np.allclose(out[14:27, 14:27], np.outer(w, w))     # and spread as the separable kernel


def light_above(height=10.0, W=64, H=48, fov_deg=90.0, k=0.8, r0=0.0):
    centre = np.array([1.0, -2.0, height])
    c2w = look_at(centre, centre - np.array([0.0, 0.0, 1.0]), up=(0.0, 1.0, 0.0))
    f = 0.5 * W / math.tan(math.radians(fov_deg) / 2)
    return OL.Light(W, H, (f, f, W / 2, H / 2), c2w, 0.0, (0.6, 0.5, 0.4), (0.1, 0.2, 0.3), k, r0)


def test_projection_and_sampling():
    L = light_above()
    c2w = np.asarray(L.c2w).reshape(3, 4)
    R, C = c2w[:, :3], c2w[:, 3]
    # points given in the light's camera frame map to fx x / z + cx
    xc = np.array([[0.0, 0.0, 4.0], [1.0, -0.5, 2.0], [-3.0, 2.0, 6.0], [0.0, 0.0, -1.0]])
    q = xc @ R.T + C
    u, v, front = OL.project(L, q)
    fx, fy, cx, cy = L.intr
    assert np.allclose(u[:3], fx * xc[:3, 0] / xc[:3, 2] + cx) and np.allclose(v[:3], fy * xc[:3, 1] / xc[:3, 2] + cy)
    assert front.tolist() == [True, True, True, False]
    img = np.arange(12.0).reshape(3, 4)
    # pixel centres give the pixel; half way between two centres gives the mean
    assert OL.sample_bilinear(img, np.array([2.5]), np.array([1.5]))[0] == img[1, 2]
    assert OL.sample_bilinear(img, np.array([2.0]), np.array([1.5]))[0] == 0.5 * (img[1, 1] + img[1, 2])
    # edge clamp inside the image, zero outside it
    assert OL.sample_bilinear(img, np.array([0.2]), np.array([0.1]))[0] == img[0, 0]
    assert OL.sample_bilinear(img, np.array([4.5, -0.1]), np.array([1.0, 1.0])).tolist() == [0.0, 0.0]


def test_shade_ground_background_and_shadow():
    L = light_above(k=0.8)
    # viewer rays from (0, 0, 3): straight down hits the ground at (0, 0, 0); straight up misses
    o = np.array([[0.0, 0.0, 3.0], [0.0, 0.0, 3.0], [50.0, 50.0, 3.0]])
    d = np.array([[0.0, 0.0, -2.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    rgb = np.zeros((3, 3))
    alpha = np.zeros(3)
    depth = np.full(3, np.inf)
    out = OL.shade(L, None, o, d, rgb, alpha, depth)
    assert np.allclose(out[0], L.ground_rgb) and np.allclose(out[1], L.background_rgb)
    # full shadow map: ground points inside the light's view are darkened by 1 - k;
    # (50, 50, 0) lies outside a 90-degree cone from 10 units up
    out = OL.shade(L, np.ones((L.height, L.width)), o, d, rgb, alpha, depth)
    assert np.allclose(out[0], 0.2 * np.asarray(L.ground_rgb))
    assert np.allclose(out[2], L.ground_rgb)
    # a shadow map with one dark pixel darkens exactly the ground point under it
    sm = np.zeros((L.height, L.width))
    sm[10, 20] = 1.0
    c2w = np.asarray(L.c2w).reshape(3, 4)
    fx, fy, cx, cy = L.intr
    xc = np.array([(20.5 - cx) / fx, (10.5 - cy) / fy, 1.0]) * 10.0      # that pixel centre, 10 below
    g = c2w[:, :3] @ xc + c2w[:, 3]
    assert abs(g[2]) < 1e-12
    oo = np.array([[g[0], g[1], 5.0], [g[0] + 0.7, g[1], 5.0]])
    dd = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    out = OL.shade(L, sm, oo, dd, np.zeros((2, 3)), np.zeros(2), np.full(2, np.inf))
    assert np.allclose(out[0], 0.2 * np.asarray(L.ground_rgb)) and np.allclose(out[1], L.ground_rgb)


def test_shade_falloff_over_and_occlusion():
    L = light_above(height=10.0, k=0.0, r0=2.0)
    C = np.asarray(L.c2w).reshape(3, 4)[:, 3]
    # performer points at distance 5 and 1 from the light along viewer rays
    o = np.array([C + [0.0, 8.0, -3.0], C + [0.0, 4.0, 0.0]])
    p = np.array([C + [0.0, 3.0, -4.0], C + [0.0, 1.0, 0.0]])                # |p - C| = 5, 1
    d = (p - o) * 0.5                                                    # not unit: depth is world distance
    depth = np.linalg.norm(p - o, axis=1)
    rgb = np.array([[0.3, 0.2, 0.1], [0.4, 0.4, 0.4]])
    alpha = np.array([0.6, 1.0])
    out = OL.shade(L, None, o, d, rgb, alpha, depth)
    # ray 0 meets the ground after the performer: performer (x (2/5)^2) over ground
    assert np.allclose(out[0], rgb[0] * (2.0 / 5.0) ** 2 + 0.4 * np.asarray(L.ground_rgb))
    # ray 1 never meets the ground (it runs parallel to it): r < r0 keeps full brightness
    assert np.allclose(out[1], rgb[1])
    # the ground met before the performer hides it
    o2 = np.array([[0.0, 0.0, 1.0]])
    d2 = np.array([[0.0, 0.0, -1.0]])
    out = OL.shade(L, None, o2, d2, np.array([[0.9, 0.9, 0.9]]), np.array([1.0]), np.array([2.0]))
    assert np.allclose(out[0], L.ground_rgb)
