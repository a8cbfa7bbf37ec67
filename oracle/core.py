"""Python front end of the FP64 oracle.

TEST INFRASTRUCTURE ONLY: used by tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; the product never imports it.

* ``render`` / ``render_grad``: the FP64 C renderer in ``render.c`` (Sec. 4.3,
  Eq. 4, 5, 8, 9, 13) through ctypes.
* ``pinhole_rays``: FP64 pinhole rays rounded once to float.
* ``compose`` / ``compose_grad``: depth-aware alpha blending (Alg. 1) in numpy,
  read as a per-pixel depth sort followed by premultiplied "over"
  (ties: the later layer is in front, as ``D_i <= D`` selects it in Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "render.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile render.c with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_render.restype = ctypes.c_int
        lib.oracle_render.argtypes = [ctypes.c_int, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int, P, P,
                                      ctypes.c_int, P, P, ctypes.c_int, P, P, P, P, P, ctypes.c_int64, P, P, P,
                                      ctypes.c_double, ctypes.c_double, P, P,
                                      P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int, P, P, ctypes.c_int,
                                      ctypes.c_int]
        lib.oracle_pinhole_rays.restype = None
        lib.oracle_pinhole_rays.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int64, P, P, P]
        lib.oracle_hh_basis.restype = None
        lib.oracle_hh_basis.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P]
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def default_threads() -> int:
    """Every CPU this process may use: its affinity set, bounded by OMP_NUM_THREADS when the
    environment sets it (a GPU host may allot each GPU a share of its cores that way)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def host_description() -> dict:
    """CPU model, online CPUs, the affinity set and the OpenMP limit of this host."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def hh_basis_c(K: int, dirs: np.ndarray, gam: np.ndarray) -> np.ndarray:
    """The C oracle's HH basis (same definition as oracle.hh, separate code)."""
    lib = _load()
    dirs = _c(dirs, np.float64).reshape(-1, 3)
    gam = _c(gam, np.float64).reshape(-1)
    out = np.zeros((dirs.shape[0], K), np.float64)
    lib.oracle_hh_basis(K, dirs.shape[0], _p(dirs), _p(gam), _p(out))
    return out


@dataclass
class Instance:
    """Spatial affine + re-timing of one placed tree (Eq. 13): local point
    R^T (x - trans) / scale; local time t + time_offset, wrapped into [0,T)
    when ``wrap`` else clamped into [0,T-1]."""
    rot: np.ndarray            # [3,3] float32 rotation
    trans: np.ndarray          # [3] float32
    scale: float = 1.0
    time_offset: float = 0.0
    wrap: bool = False

    def packed(self) -> np.ndarray:
        v = np.zeros(15, np.float64)
        v[:9] = np.asarray(self.rot, np.float32).astype(np.float64).reshape(-1)
        v[9:12] = np.asarray(self.trans, np.float32).astype(np.float64)
        v[12] = float(np.float32(self.scale))
        v[13] = float(np.float32(self.time_offset))
        v[14] = 1.0 if self.wrap else 0.0
        return v


def render(depth: int, leaf_ijk, hh, wsig, basis, gamma, ray_o, ray_d, ray_t=None, t_scalar=0.0,
           t_stop=1e-4, inst: Optional[Instance] = None, g_rgb=None, g_alpha=None,
           want_grad_basis=True, threads: Optional[int] = None, wgam=None, basis_g=None, edit=None,
           segments: bool = False, density: str = "softplus"):
    """FP64 render of float32 rays through a tree given by its leaf cells.

    leaf_ijk [N,3] int; hh [N,3,K]; wsig [N,C]; basis [T,C]; gamma [T] (all as
    the exact values the product stores: pass dtype-rounded arrays for 16-bit
    storage). With wgam [N,Cg] and basis_g [T,Cg] the hyperangle is per point,
    gamma = pi sigmoid(sum_c wgam_c basis_g_c(t)) (Eq. 6), and gamma is unused.
    Returns a dict with rgb [n,3], alpha, depth, nsamp, tfinal, margin [n,2]
    (smallest sampled segment length, smallest relative distance of T to t_stop
    at a stop test) and, if g_rgb is given, grad_hh [N,3,K], grad_wsig [N,C],
    grad_basis [T,C] (and grad_wgam [N,Cg], grad_basis_g [T,Cg]) of
    <g_rgb, rgb> + <g_alpha, alpha>, and last_leaf [n]: the input index of the
    leaf of a ray's last sample when the ray stopped (T < t_stop), else -1.
    With segments=True also seg [n, cap, 6] (every composited sample's ray interval
    [u_in, u_out), density per leaf unit and colour; nsamp[r] rows valid) and len [n]
    (leaf units per unit of the ray parameter).
    edit [N,5] (target rgb, target density or < 0 to keep it, first frame t_d)
    replaces a leaf's colour (and density) at local times tau >= t_d, the
    appearance edit of Sec. 5.2; no gradient is taken with edits.
    density: the activation of Eq. 5, "softplus" (the workloads' reading) or "relu" (as Eq. 5
    prints it; derivative 0 at a logit of exactly 0).
    """
    if density not in ("softplus", "relu"):
        raise ValueError(f"unknown density activation {density!r}")
    lib = _load()
    leaf_ijk = _c(leaf_ijk, np.int32).reshape(-1, 3)
    hh = _c(hh, np.float64)
    N, three, K = hh.shape
    assert three == 3 and leaf_ijk.shape[0] == N
    wsig = _c(wsig, np.float64)
    C = wsig.shape[1]
    basis = _c(basis, np.float64)
    T = basis.shape[0]
    gamma = _c(gamma, np.float64).reshape(-1)
    ray_o = _c(ray_o, np.float32).reshape(-1, 3)
    ray_d = _c(ray_d, np.float32).reshape(-1, 3)
    n = ray_o.shape[0]
    ray_t = None if ray_t is None else _c(ray_t, np.float32).reshape(-1)
    ip = None if inst is None else inst.packed()
    Cg = 0
    if wgam is not None:
        wgam = _c(wgam, np.float64)
        basis_g = _c(basis_g, np.float64)
        Cg = wgam.shape[1]
        assert wgam.shape[0] == N and basis_g.shape == (T, Cg)
    out = dict(rgb=np.zeros((n, 3)), alpha=np.zeros(n), depth=np.zeros(n),
               nsamp=np.zeros(n, np.int32), tfinal=np.zeros(n), margin=np.zeros((n, 2)),
               last_leaf=np.full(n, -1, np.int64))
    if edit is not None:
        edit = _c(edit, np.float64).reshape(N, 5)
    cap = 0
    if segments:
        cap = 3 * (1 << depth) + 8
        out["seg"] = np.zeros((n, cap, 6))
        out["len"] = np.zeros(n)
    gr = ga = None
    if g_rgb is not None:
        gr = _c(g_rgb, np.float64).reshape(-1, 3)
        ga = None if g_alpha is None else _c(g_alpha, np.float64).reshape(-1)
        out["grad_hh"] = np.zeros((N, 3, K))
        out["grad_wsig"] = np.zeros((N, C))
        out["grad_basis"] = np.zeros((T, C)) if want_grad_basis else None
        if wgam is not None:
            out["grad_wgam"] = np.zeros((N, Cg))
            out["grad_basis_g"] = np.zeros((T, Cg)) if want_grad_basis else None
    rc = lib.oracle_render(depth, N, _p(leaf_ijk), K, C, _p(hh), _p(wsig), T, _p(basis), _p(gamma),
                           Cg, _p(wgam), _p(basis_g), _p(out.get("grad_wgam")), _p(out.get("grad_basis_g")),
                           _p(ip), n, _p(ray_o), _p(ray_d), _p(ray_t), float(t_scalar), float(t_stop),
                           _p(gr), _p(ga), _p(out["rgb"]), _p(out["alpha"]), _p(out["depth"]),
                           _p(out["nsamp"]), _p(out["tfinal"]), _p(out["margin"]),
                           _p(out.get("grad_hh")), _p(out.get("grad_wsig")), _p(out.get("grad_basis")),
                           _p(edit), _p(out["last_leaf"]), int(cap), _p(out.get("seg")), _p(out.get("len")),
                           1 if density == "relu" else 0, int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError(f"oracle_render failed with code {rc}")
    return out


def pinhole_rays(W: int, H: int, intr, c2w, pix=None):
    """FP64 pinhole rays rounded once to float32: (ray_o [n,3], ray_d [n,3])."""
    lib = _load()
    intr = _c(np.asarray(intr, np.float32), np.float64)
    c2w = _c(np.asarray(c2w, np.float32).reshape(12), np.float64)
    pix = None if pix is None else _c(pix, np.int32).reshape(-1)
    n = W * H if pix is None else pix.shape[0]
    o = np.zeros((n, 3), np.float32)
    d = np.zeros((n, 3), np.float32)
    lib.oracle_pinhole_rays(W, H, _p(intr), _p(c2w), n, _p(pix), _p(o), _p(d))
    return o, d


# ---------------------------------------------------------------------------
# depth-aware alpha blending (Alg. 1), read as sort + premultiplied over

def _order(depth: np.ndarray) -> np.ndarray:
    """Per pixel, layer indices front to back: ascending depth, ties -> later layer first."""
    L, n = depth.shape
    lay = np.broadcast_to(np.arange(L)[:, None], (L, n))
    # lexsort: last key is primary. Sort by depth ascending, then by -layer.
    keys = (-lay, depth)
    return np.lexsort(keys, axis=0)


def compose(rgb, alpha, depth):
    """rgb [L,n,3] premultiplied, alpha [L,n], depth [L,n] -> (rgb [n,3], alpha [n], depth [n])."""
    rgb = np.asarray(rgb, np.float64)
    alpha = np.asarray(alpha, np.float64)
    depth = np.asarray(depth, np.float64)
    L, n = alpha.shape
    order = _order(depth)
    cols = np.arange(n)
    out = np.zeros((n, 3))
    M = np.ones(n)
    for k in range(L):
        idx = order[k]
        out += M[:, None] * rgb[idx, cols]
        M = M * (1.0 - alpha[idx, cols])
    return out, 1.0 - M, depth[order[0], cols]


def compose_grad(rgb, alpha, depth, g_rgb, g_alpha):
    """Gradient of <g_rgb, out_rgb> + <g_alpha, out_alpha> w.r.t. every layer's
    rgb [L,n,3] and alpha [L,n]; depth is a sort key and carries none."""
    rgb = np.asarray(rgb, np.float64)
    alpha = np.asarray(alpha, np.float64)
    g_rgb = np.asarray(g_rgb, np.float64)
    g_alpha = np.asarray(g_alpha, np.float64)
    L, n = alpha.shape
    order = _order(np.asarray(depth, np.float64))
    cols = np.arange(n)
    Ps = [rgb[order[k], cols] for k in range(L)]
    As = [alpha[order[k], cols] for k in range(L)]
    M = [np.ones(n)]
    for k in range(L):
        M.append(M[-1] * (1.0 - As[k]))
    # suffix composites S_k = P_k + (1-A_k) S_{k+1}; suffix transmittance Q_k = prod_{i>=k}(1-A_i)
    S = [None] * (L + 1)
    Q = [None] * (L + 1)
    S[L] = np.zeros((n, 3))
    Q[L] = np.ones(n)
    for k in range(L - 1, -1, -1):
        S[k] = Ps[k] + (1.0 - As[k])[:, None] * S[k + 1]
        Q[k] = Q[k + 1] * (1.0 - As[k])
    gP = np.zeros_like(rgb)
    gA = np.zeros_like(alpha)
    for k in range(L):
        idx = order[k]
        gP[idx, cols] = M[k][:, None] * g_rgb
        gA[idx, cols] = -M[k] * np.sum(g_rgb * S[k + 1], axis=1) + g_alpha * M[k] * Q[k + 1]
    return gP, gA
