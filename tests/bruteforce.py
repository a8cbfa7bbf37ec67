"""Brute-force FP64 references used to pin the oracle (tiny inputs only).

* ``segments``: every crossing of the ray with every integer plane of the
  grid, sorted; each interval between consecutive crossings is classified by
  its midpoint against a dense occupancy grid. No DDA, no hashing.
* ``render``: Eq. 8 written literally, T_i = exp(-sum_{j<i} sigma_j delta_j),
  over those segments, with the early stop after the first sample whose
  following transmittance is below t_stop.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.hh import hh_basis


def segments(depth, occ, o, d):
    """occ: dense bool grid [G,G,G] indexed [i,j,k]. o, d float64 local ray.
    Returns a list of (i,j,k, u0, u1) for occupied cells in increasing u."""
    G = 1 << depth
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    if not np.any(d != 0):
        return []
    us = [0.0]
    for a in range(3):
        if d[a] != 0:
            for k in range(G + 1):
                u = (k - o[a]) / d[a]
                if u > 0:
                    us.append(u)
    us = sorted(set(us))
    out = []
    for u0, u1 in zip(us[:-1], us[1:]):
        m = 0.5 * (u0 + u1)
        p = o + m * d
        if np.all(p >= 0) and np.all(p < G):
            c = np.floor(p).astype(int)
            if occ[c[0], c[1], c[2]]:
                out.append((c[0], c[1], c[2], u0, u1))
    # a ray lying in a cell face belongs to the cell on the + side (half-open cells);
    # the midpoint classification above already does that through floor().
    return out


def softplus(x):
    return max(x, 0.0) + math.log1p(math.exp(-abs(x)))


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def render(depth, leaf_ijk, hh, wsig, basis, gamma, o, d, t, t_stop, wgam=None, basis_g=None, density="softplus"):
    """Single identity-instance ray, t an exact frame index or fraction in [0, T-1].
    With wgam/basis_g the hyperangle of each sample is pi * sigmoid(wgam . basis_g(t)) (Eq. 6).
    density: "softplus" or "relu" (Eq. 5 as printed)."""
    G = 1 << depth
    occ = np.zeros((G, G, G), bool)
    idx = -np.ones((G, G, G), np.int64)
    for q, (i, j, k) in enumerate(leaf_ijk):
        occ[i, j, k] = True
        idx[i, j, k] = q
    T = basis.shape[0]
    i0 = int(math.floor(t))
    f = t - i0
    i1 = min(i0 + 1, T - 1)
    if i0 == T - 1:
        f = 0.0
    b = (1 - f) * basis[i0].astype(np.float64) + f * basis[i1].astype(np.float64)
    gam = (1 - f) * float(gamma[i0]) + f * float(gamma[i1])
    d = np.asarray(d, np.float64)
    n = np.linalg.norm(d)
    K = hh.shape[2]
    h = hh_basis(K, d / n if n > 0 else np.array([0, 0, 1.0]), gam) if n > 0 else None
    segs = segments(depth, occ, o, d)
    sig_del = []
    cols = []
    mids = []
    if wgam is not None:
        bg = (1 - f) * basis_g[i0].astype(np.float64) + f * basis_g[i1].astype(np.float64)
    for (i, j, k, u0, u1) in segs:
        q = idx[i, j, k]
        if wgam is not None:
            gq = math.pi * sigmoid(float(np.dot(wgam[q].astype(np.float64), bg)))
            h = hh_basis(K, d / n, gq)
        x = float(np.dot(wsig[q].astype(np.float64), b))
        sig = max(x, 0.0) if density == "relu" else softplus(x)
        c = np.array([sigmoid(float(np.dot(hh[q, ch].astype(np.float64), h))) for ch in range(3)])
        sig_del.append(sig * (u1 - u0) * n)
        cols.append(c)
        mids.append(0.5 * (u0 + u1) * n)
    C = np.zeros(3)
    A = 0.0
    D = 0.0
    ns = 0
    for i in range(len(sig_del)):
        Ti = math.exp(-sum(sig_del[:i]))
        w = Ti * (1 - math.exp(-sig_del[i]))
        C += w * cols[i]
        A += w
        D += w * mids[i]
        ns += 1
        if t_stop > 0 and math.exp(-sum(sig_del[:i + 1])) < t_stop:
            break
    return C, A, (D / A if A > 0 else math.inf), ns
