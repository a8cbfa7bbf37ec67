"""FP64 oracle of the spotlight shadow and distance-falloff lighting (Sec. 5.2
"Spotlight Lighting", Sec. 6 "Lighting").

TEST INFRASTRUCTURE ONLY: used by tests/ and bench.py's lighting check; the
product never imports it.

The paper describes the effect, not formulas. The readings written here:

* The shadow map is the alpha map (Eq. 9) rendered from a pinhole camera
  placed at the point light, low-passed with a Gaussian to remove moire
  (``blur``): a separable kernel w_i proportional to exp(-i^2 / (2 sigma^2))
  for |i| <= round(3 sigma), normalised to sum 1, borders clamped to the edge.
* Ground shadow: a viewer ray meets the ground plane z = ground_z at q; q is
  projected into the light camera (pixel centres at +1/2) and the blurred
  alpha A is sampled bilinearly there (clamped to the edge inside the image,
  0 outside it or behind the light); the ground colour is scaled by
  1 - k A, k the shadow strength.
* Falloff: the performer's premultiplied colour at a pixel is scaled by
  (r0 / max(r, r0))^2, r the distance from the light to the pixel's expected
  surface point o + depth * d / |d| (depth as rendered, world units).
* The ground is opaque: where it is met before the performer's expected depth
  it hides the performer; elsewhere the performer is composited over it
  (premultiplied over). Rays that miss the ground see the background colour.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def gaussian_weights(sigma: float) -> np.ndarray:
    """Normalised 1-D Gaussian taps for offsets -r..r, r = round(3 sigma)."""
    r = int(3.0 * sigma + 0.5)
    i = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(i * i) / (2.0 * sigma * sigma))
    return w / w.sum()


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian low-pass of an [H, W] map, borders clamped to the edge."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    w = gaussian_weights(sigma)
    r = (len(w) - 1) // 2
    rows = np.zeros_like(img)
    for k, wk in enumerate(w):
        xs = np.clip(np.arange(W) + k - r, 0, W - 1)
        rows += wk * img[:, xs]
    out = np.zeros_like(img)
    for k, wk in enumerate(w):
        ys = np.clip(np.arange(H) + k - r, 0, H - 1)
        out += wk * rows[ys, :]
    return out


@dataclass
class Light:
    width: int
    height: int
    intr: tuple            # fx, fy, cx, cy of the light camera (pixels)
    c2w: np.ndarray        # [3, 4] camera-to-world [R | centre]; the centre is the point light
    ground_z: float
    ground_rgb: tuple
    background_rgb: tuple
    shadow_strength: float
    falloff_r0: float      # > 0 enables the falloff


def project(light: Light, q: np.ndarray):
    """World points [n, 3] -> light-image coordinates (u, v) and a visibility flag (in front)."""
    c2w = np.asarray(light.c2w, np.float64).reshape(3, 4)
    R, C = c2w[:, :3], c2w[:, 3]
    x = (np.asarray(q, np.float64) - C) @ R          # R^T (q - C), row vectors
    fx, fy, cx, cy = (float(v) for v in light.intr)
    front = x[:, 2] > 0.0
    z = np.where(front, x[:, 2], 1.0)
    return fx * x[:, 0] / z + cx, fy * x[:, 1] / z + cy, front


def sample_bilinear(img: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Bilinear sample at image coordinates (pixel centres at +1/2), edge-clamped inside the
    image rectangle [0, W] x [0, H]; 0 outside it."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    inside = (u >= 0.0) & (u <= W) & (v >= 0.0) & (v <= H)
    x, y = u - 0.5, v - 0.5
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = x - x0, y - y0
    xi0 = np.clip(x0, 0, W - 1).astype(np.int64)
    xi1 = np.clip(x0 + 1, 0, W - 1).astype(np.int64)
    yi0 = np.clip(y0, 0, H - 1).astype(np.int64)
    yi1 = np.clip(y0 + 1, 0, H - 1).astype(np.int64)
    val = ((1 - fy) * ((1 - fx) * img[yi0, xi0] + fx * img[yi0, xi1]) +
           fy * ((1 - fx) * img[yi1, xi0] + fx * img[yi1, xi1]))
    return np.where(inside, val, 0.0)


def shade(light: Light, shadow_map, ray_o, ray_d, rgb, alpha, depth) -> np.ndarray:
    """Viewer image [n, 3] of a rendered performer layer (premultiplied rgb, alpha, depth) over
    the lit ground, with the shadow map (blurred light alpha, or None) and the falloff."""
    o = np.asarray(ray_o, np.float64)
    d = np.asarray(ray_d, np.float64)
    rgb = np.asarray(rgb, np.float64)
    alpha = np.asarray(alpha, np.float64)
    depth = np.asarray(depth, np.float64)
    dn = np.linalg.norm(d, axis=1)
    centre = np.asarray(light.c2w, np.float64).reshape(3, 4)[:, 3]
    # falloff of the performer's colour
    F = np.ones(o.shape[0])
    if light.falloff_r0 > 0.0:
        ok = np.isfinite(depth) & (dn > 0)
        p = o + (np.where(ok, depth, 0.0) / np.where(dn > 0, dn, 1.0))[:, None] * d
        r = np.linalg.norm(p - centre, axis=1)
        F = np.where(ok, (light.falloff_r0 / np.maximum(r, light.falloff_r0)) ** 2, 1.0)
    perf = rgb * F[:, None]
    # ground hit
    dz = d[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(dz != 0.0, (light.ground_z - o[:, 2]) / dz, -1.0)
    hit = t > 0.0
    q = o + np.where(hit, t, 0.0)[:, None] * d
    S = np.zeros(o.shape[0])
    if shadow_map is not None:
        u, v, front = project(light, q)
        S = np.where(front & hit, sample_bilinear(shadow_map, u, v), 0.0)
    ground = np.asarray(light.ground_rgb, np.float64)[None, :] * (1.0 - light.shadow_strength * S)[:, None]
    bg = np.broadcast_to(np.asarray(light.background_rgb, np.float64), ground.shape)
    G = np.where(hit[:, None], ground, bg)
    ground_first = hit & (t * dn < depth)
    out = perf + (1.0 - alpha)[:, None] * G
    return np.where(ground_first[:, None], G, out)
