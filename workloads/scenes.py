"""Seeded synthetic VOctree scenes, cameras and ray sets.

The paper's captured performers (66 cameras, 3840x2160, 75-150 frames) are not
available, so every scene is a synthetic stand-in with their shape: a
human-sized union of ellipsoids filling a few per cent of its bounding cube,
leaf payloads of K hyperspherical-harmonic coefficients per colour channel and
C density weights, a shared density basis over T frames and a hyperangle table.

Nothing here renders: these are inputs only. Both the FP64 oracle and the GPU
path receive exactly these arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = ["Scene", "Camera", "Ellipsoid", "WORKLOADS", "make_scene", "make_scene_per_point", "make_payload",
           "scene_for_workload",
           "look_at", "ring_cameras", "orbit_camera", "random_rays", "special_rays", "stereo_cameras",
           "multi_instances", "random_rotation", "humanoid_ellipsoids", "random_ellipsoids",
           "occupancy_from_ellipsoids", "default_gamma"]


@dataclass
class Ellipsoid:
    centre: np.ndarray   # [3] grid units
    radii: np.ndarray    # [3] grid units
    rot: np.ndarray      # [3,3], columns are the ellipsoid axes in grid coordinates


@dataclass
class Scene:
    depth: int
    leaf_ijk: np.ndarray          # [N,3] int32 occupied leaf cells, sorted by i + G (j + G k)
    hh: np.ndarray                # [N,3,K] float32 HH coefficients per colour channel
    wsig: np.ndarray              # [N,C] float32 density weights
    basis: np.ndarray             # [T,C] float32 shared density basis (row t = frame t)
    gamma: np.ndarray             # [T] float32 hyperangle per frame
    seed: int = 0
    meta: Dict = field(default_factory=dict)
    wgam: Optional[np.ndarray] = None     # [N,Cg] float32 per-point hyperangle weights, or None
    basis_g: Optional[np.ndarray] = None  # [T,Cg] float32 hyperangle basis, or None

    @property
    def G(self) -> int:
        return 1 << self.depth

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_ijk.shape[0])

    @property
    def K(self) -> int:
        return int(self.hh.shape[2])

    @property
    def C(self) -> int:
        return int(self.wsig.shape[1])

    @property
    def T(self) -> int:
        return int(self.basis.shape[0])


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    c2w: np.ndarray               # [3,4] float32, OpenCV axes (x right, y down, z forward)

    def intr(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], np.float32)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


# ---------------------------------------------------------------------------
# occupancy

def random_rotation(rng: np.random.Generator, max_angle: Optional[float] = None) -> np.ndarray:
    """Uniform random rotation, or a rotation about a random axis by at most max_angle rad."""
    if max_angle is None:
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                         [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                         [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    ang = rng.uniform(-max_angle, max_angle)
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + math.sin(ang) * Kx + (1 - math.cos(ang)) * (Kx @ Kx)


# Humanoid template in units of the cube edge: (name, centre, radii, tilt about y in degrees).
_HUMANOID = [
    ("head", (0.50, 0.50, 0.885), (0.060, 0.068, 0.080), 0.0),
    ("neck", (0.50, 0.50, 0.795), (0.034, 0.034, 0.040), 0.0),
    ("torso", (0.50, 0.50, 0.640), (0.130, 0.080, 0.140), 0.0),
    ("pelvis", (0.50, 0.50, 0.480), (0.120, 0.075, 0.070), 0.0),
    ("upper_arm_l", (0.33, 0.50, 0.660), (0.040, 0.040, 0.110), 12.0),
    ("upper_arm_r", (0.67, 0.50, 0.660), (0.040, 0.040, 0.110), -12.0),
    ("forearm_l", (0.295, 0.50, 0.455), (0.035, 0.035, 0.100), 5.0),
    ("forearm_r", (0.705, 0.50, 0.455), (0.035, 0.035, 0.100), -5.0),
    ("thigh_l", (0.435, 0.50, 0.340), (0.055, 0.055, 0.130), 3.0),
    ("thigh_r", (0.565, 0.50, 0.340), (0.055, 0.055, 0.130), -3.0),
    ("shin_l", (0.430, 0.50, 0.120), (0.045, 0.045, 0.120), 0.0),
    ("shin_r", (0.570, 0.50, 0.120), (0.045, 0.045, 0.120), 0.0),
]


def _rot_y(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])


def humanoid_ellipsoids(G: int, rng: np.random.Generator) -> List[Ellipsoid]:
    """12 jittered ellipsoids (head, neck, torso, pelvis, arms, legs); vertical axis = z.
    Jitter: centres +-2 % of G, radii x U[0.9,1.1], tilts up to 10 degrees."""
    out = []
    for _, c, r, tilt in _HUMANOID:
        centre = np.asarray(c) * G + rng.uniform(-0.02, 0.02, 3) * G
        radii = np.asarray(r) * G * rng.uniform(0.9, 1.1, 3)
        rot = random_rotation(rng, math.radians(10.0)) @ _rot_y(tilt)
        out.append(Ellipsoid(centre, radii, rot))
    return out


def random_ellipsoids(G: int, n: int, rng: np.random.Generator) -> List[Ellipsoid]:
    out = []
    for _ in range(n):
        centre = rng.uniform(0.3, 0.7, 3) * G
        radii = rng.uniform(0.10, 0.25, 3) * G
        out.append(Ellipsoid(centre, radii, random_rotation(rng)))
    return out


def occupancy_from_ellipsoids(depth: int, ells: List[Ellipsoid], factor: float = 1.0) -> np.ndarray:
    """Cells (i,j,k) of [0,2^depth)^3 whose centre lies inside any ellipsoid with radii x factor.
    Returned sorted by the key i + G (j + G k)."""
    G = 1 << depth
    keys = []
    for e in ells:
        r = e.radii * factor
        half = np.sqrt(((e.rot * r[None, :]) ** 2).sum(axis=1))
        lo = np.clip(np.floor(e.centre - half - 0.5).astype(np.int64), 0, G - 1)
        hi = np.clip(np.ceil(e.centre + half + 0.5).astype(np.int64), 0, G - 1)
        xs = np.arange(lo[0], hi[0] + 1)
        ys = np.arange(lo[1], hi[1] + 1)
        inv = e.rot / r[None, :]        # maps offset p - c to ellipsoid-normalised coordinates
        for z0 in range(lo[2], hi[2] + 1, 16):
            zs = np.arange(z0, min(z0 + 16, hi[2] + 1))
            X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
            P = np.stack([X, Y, Z], -1).astype(np.float64) + 0.5 - e.centre
            q = P @ inv
            m = (q * q).sum(-1) <= 1.0
            if m.any():
                keys.append(X[m] + G * (Y[m] + G * Z[m].astype(np.int64)))
    if not keys:
        return np.zeros((0, 3), np.int32)
    k = np.unique(np.concatenate(keys))
    ijk = np.stack([k % G, (k // G) % G, k // (G * G)], -1)
    return ijk.astype(np.int32)


def _fit_occupancy(depth: int, ells: List[Ellipsoid], target: int, tol: float = 0.02) -> Tuple[np.ndarray, float]:
    # start from the radius factor at which the summed ellipsoid volumes equal the target
    vol = sum(4.0 / 3.0 * math.pi * float(np.prod(e.radii)) for e in ells)
    f = min(1.0, (target / max(vol, 1e-30)) ** (1.0 / 3.0))
    ijk = occupancy_from_ellipsoids(depth, ells, f)
    for _ in range(8):
        n = ijk.shape[0]
        if n > 0 and abs(n - target) <= tol * target:
            break
        f *= (target / max(n, 1)) ** (1.0 / 3.0)
        ijk = occupancy_from_ellipsoids(depth, ells, f)
    return ijk, f


def default_gamma(T: int) -> np.ndarray:
    """Hyperangle table gamma(t) = pi (t + 1/2) / T spread over (0, pi)."""
    return (math.pi * (np.arange(T) + 0.5) / T).astype(np.float32)


def make_payload(n_leaves: int, K: int, C: int, T: int, rng: np.random.Generator):
    """Leaf payload in leaf order: hh ~ N(0, 0.3) [N,3,K], wsig ~ N(0,1) [N,C]; basis ~ N(0,1) [T,C]."""
    hh = rng.normal(0.0, 0.3, size=(n_leaves, 3, K)).astype(np.float32)
    wsig = rng.normal(0.0, 1.0, size=(n_leaves, C)).astype(np.float32)
    basis = rng.normal(0.0, 1.0, size=(T, C)).astype(np.float32)
    return hh, wsig, basis


def make_scene(depth: int, target_leaves: int, kind: str = "human", K: int = 16, C: int = 8, T: int = 300,
               seed: int = 0, n_random: int = 3) -> Scene:
    """Occupancy first, then payload, from one PCG64 stream seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    G = 1 << depth
    ells = humanoid_ellipsoids(G, rng) if kind == "human" else random_ellipsoids(G, n_random, rng)
    ijk, f = _fit_occupancy(depth, ells, target_leaves)
    hh, wsig, basis = make_payload(ijk.shape[0], K, C, T, rng)
    return Scene(depth, ijk, hh, wsig, basis, default_gamma(T), seed,
                 dict(kind=kind, radius_factor=f, target=target_leaves, ellipsoids=ells))


def make_scene_per_point(depth: int, target_leaves: int, kind: str = "human", T: int = 300, seed: int = 0,
                         K: int = 14, C: int = 31, Cg: int = 31, n_random: int = 3) -> Scene:
    """The paper's full leaf (K = 14 HH per channel, C = 31 density weights, Cg = 31
    hyperangle weights). Occupancy and payload draws as make_scene, then wgam ~ N(0, 0.2)
    [N,Cg] and basis_g ~ N(0,1) [T,Cg] from the same stream. The density weights are drawn
    with standard deviation sqrt(8 / C), so that the density logit has the spread it has with
    C = 8 (the optical depth per leaf of the other workloads)."""
    rng = np.random.default_rng(seed)
    G = 1 << depth
    ells = humanoid_ellipsoids(G, rng) if kind == "human" else random_ellipsoids(G, n_random, rng)
    ijk, f = _fit_occupancy(depth, ells, target_leaves)
    hh, wsig, basis = make_payload(ijk.shape[0], K, C, T, rng)
    wsig = (wsig * np.float32(math.sqrt(8.0 / C))).astype(np.float32)
    wgam = rng.normal(0.0, 0.2, size=(ijk.shape[0], Cg)).astype(np.float32)
    basis_g = rng.normal(0.0, 1.0, size=(T, Cg)).astype(np.float32)
    return Scene(depth, ijk, hh, wsig, basis, default_gamma(T), seed,
                 dict(kind=kind, radius_factor=f, target=target_leaves, ellipsoids=ells, per_point=True),
                 wgam, basis_g)


# The five workloads by name (depth, target leaves, kind, K, C, T, seed): tiny (depth 6, ~20k random
# leaves), forward (depth-9 humanoid, ~2M leaves), train (depth 8, ~500k), mixed (depth 10, ~8M) and
# multi (depth-9 primitives placed four times).
WORKLOADS = {
    "tiny": dict(depth=6, target=20_000, kind="random", K=16, C=8, T=30, seed=1),
    "forward": dict(depth=9, target=2_000_000, kind="human", K=16, C=8, T=300, seed=2),
    "train": dict(depth=8, target=500_000, kind="human", K=16, C=8, T=300, seed=3),
    "mixed": dict(depth=10, target=8_000_000, kind="human", K=16, C=8, T=300, seed=4),
    "multi": dict(depth=9, target=2_000_000, kind="human", K=16, C=8, T=300, seed=50),
}


def scene_for_workload(name: str, depth: Optional[int] = None, target: Optional[int] = None,
                       seed: Optional[int] = None) -> Scene:
    c = WORKLOADS[name]
    d = c["depth"] if depth is None else depth
    if target is None:
        target = c["target"] if depth is None else max(64, int(c["target"] * 8.0 ** (d - c["depth"])))
    return make_scene(d, target, c["kind"], c["K"], c["C"], c["T"], c["seed"] if seed is None else seed)


# ---------------------------------------------------------------------------
# cameras and rays

def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """3x4 camera-to-world matrix, OpenCV axes: x right, y down, z forward."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(r) < 1e-9:
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    m = np.zeros((3, 4))
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = r, dn, f, eye
    return m.astype(np.float32)


def _intrinsics(W: int, H: int, hfov_deg: float):
    fx = (W / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return float(np.float32(fx)), float(np.float32(fx)), W / 2.0, H / 2.0


def orbit_camera(centre, dist, azim, elev, W, H, hfov_deg) -> Camera:
    centre = np.asarray(centre, np.float64)
    eye = centre + dist * np.array([math.cos(elev) * math.cos(azim), math.cos(elev) * math.sin(azim),
                                    math.sin(elev)])
    fx, fy, cx, cy = _intrinsics(W, H, hfov_deg)
    return Camera(W, H, fx, fy, cx, cy, look_at(eye, centre))


def _bbox(scene: Scene):
    lo = scene.leaf_ijk.min(0).astype(np.float64)
    hi = scene.leaf_ijk.max(0).astype(np.float64) + 1.0
    return lo, hi


def ring_cameras(scene: Scene, n: int, W: int, H: int, hfov_deg: float = 40.0, elev_deg: float = 10.0,
                 fill: float = 0.8, seed: int = 0) -> List[Camera]:
    """n cameras on a ring around the occupied box, the blob spanning about ``fill`` of the image height."""
    rng = np.random.default_rng(seed)
    lo, hi = _bbox(scene)
    centre = 0.5 * (lo + hi)
    fx, fy, _, _ = _intrinsics(W, H, hfov_deg)
    dist = fy * (hi[2] - lo[2]) / (fill * H) + 0.5 * max(hi[0] - lo[0], hi[1] - lo[1])
    phase = rng.uniform(0, 2 * math.pi)
    return [orbit_camera(centre, dist, phase + 2 * math.pi * i / n, math.radians(elev_deg), W, H, hfov_deg)
            for i in range(n)]


def stereo_cameras(scene: Scene, W: int, H: int, hfov_deg: float = 90.0, seed: int = 0,
                   dist_factor: float = 1.6) -> List[Camera]:
    """Left/right eye pinholes, IPD = 0.064 x (blob height / 1.7), looking at the blob."""
    rng = np.random.default_rng(seed)
    lo, hi = _bbox(scene)
    centre = 0.5 * (lo + hi)
    height = hi[2] - lo[2]
    ipd = 0.064 * height / 1.7
    az = rng.uniform(0, 2 * math.pi)
    dist = dist_factor * height
    eye_c = centre + dist * np.array([math.cos(az), math.sin(az), 0.05])
    fwd = centre - eye_c
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    fx, fy, cx, cy = _intrinsics(W, H, hfov_deg)
    cams = []
    for s in (-0.5, 0.5):
        eye = eye_c + s * ipd * right
        cams.append(Camera(W, H, fx, fy, cx, cy, look_at(eye, eye + fwd * dist)))
    return cams


def random_rays(G: int, n: int, rng: np.random.Generator, inside_frac: float = 0.1):
    """Float32 rays: origins on a sphere of radius 2G around the cube centre (a fraction inside
    the cube), directions towards uniform points of the cube (not normalised)."""
    c = np.full(3, G / 2.0)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o = c + 2.0 * G * v
    k = int(n * inside_frac)
    o[:k] = rng.uniform(0, G, size=(k, 3))
    tgt = rng.uniform(0, G, size=(n, 3))
    d = tgt - o
    return o.astype(np.float32), d.astype(np.float32)


def special_rays(G: int):
    """Degenerate rays: axis-parallel (on cell centres and on cell faces), through lattice
    vertices, starting on faces, missing the cube, zero direction, negative directions."""
    o, d = [], []
    h = G / 2.0
    for a in range(3):
        for sgn in (1.0, -1.0):
            for off in (0.5, 0.0, 1.0, float(G // 2), h + 0.25):
                p = np.full(3, off if off != 0.5 else h + 0.5)
                p[(a + 1) % 3] = off
                p[a] = -3.0 if sgn > 0 else G + 3.0
                dd = np.zeros(3)
                dd[a] = sgn
                o.append(p.copy())
                d.append(dd)
    # diagonals through lattice vertices
    for dd in ((1, 1, 1), (1, -1, 1), (-1, -1, -1), (1, 1, 0), (0, 1, -1), (2, 1, 0)):
        dd = np.asarray(dd, np.float64)
        start = np.full(3, h) - 3 * G * dd / np.linalg.norm(dd)
        o.append(np.round(start))
        d.append(dd)
        o.append(np.full(3, float(G // 2)))
        d.append(dd)
    # origin on a cell face, looking both ways along that axis
    o.append(np.array([h, h, float(G // 2)])); d.append(np.array([0.0, 0.0, -1.0]))
    o.append(np.array([h, h, float(G // 2)])); d.append(np.array([0.0, 0.0, 1.0]))
    # misses: parallel outside, pointing away, exactly on the far face plane
    o.append(np.array([-1.0, h, h])); d.append(np.array([0.0, 1.0, 0.0]))
    o.append(np.array([-5.0, h, h])); d.append(np.array([-1.0, 0.0, 0.0]))
    o.append(np.array([float(G), h, h])); d.append(np.array([0.0, 1.0, 0.0]))
    # zero direction (treated as a miss)
    o.append(np.array([h, h, h])); d.append(np.zeros(3))
    return np.asarray(o, np.float32), np.asarray(d, np.float32)


def multi_instances(G: int, n: int, seed: int):
    """Seeded placements for n trees: rotation about z ~ U[0,2pi), scale ~ U[0.5,2],
    standing on the ground plane z = 0 around the origin, time offset ~ U[0,150], looping."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        th = rng.uniform(0, 2 * math.pi)
        s = rng.uniform(0.5, 2.0)
        R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
        ang = 2 * math.pi * i / n + rng.uniform(-0.3, 0.3)
        pos = 0.9 * G * np.array([math.cos(ang), math.sin(ang), 0.0])
        trans = pos - s * (R @ np.array([G / 2.0, G / 2.0, 0.0]))
        off = rng.uniform(0, 150)
        out.append(dict(rot=R.astype(np.float32), trans=trans.astype(np.float32), scale=float(np.float32(s)),
                        time_offset=float(np.float32(off)), wrap=True))
    return out
