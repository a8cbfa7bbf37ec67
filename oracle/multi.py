"""Oracle of the exact per-ray merge of several placed VOctree instances
(Sec. 5.1 composition, extended to interpenetrating primitives and duplicates).

TEST INFRASTRUCTURE ONLY: used by tests/ and bench.py's checks; the product
never imports it.

Reading: every instance k turns a world ray (o, d) into its own local ray with
the same parameter u (x_l = R_k^T (o + u d - t_k) / s_k), and its leaves give
disjoint intervals [u_in, u_out) of constant density sigma (per leaf unit) and
colour c. Along u the instances' media overlap, and volume rendering (Eq. 8)
of overlapping constant media is exact on the intervals between consecutive
boundaries of all instances: on such an interval of length du the extinction
per unit u of instance k is kappa_k = sigma_k |d_l,k| (|d_l,k| = |d| / s_k,
leaf units per unit u), the optical depth is sum_k kappa_k du, and the
emitted colour is the kappa-weighted mean of the active instances' colours.
Intervals are composited front to back with the early stop after the first
interval that leaves T < t_stop, as in the single render; nsamp counts the
composited intervals. With one instance this is exactly the single render;
with instances disjoint in depth along a ray it is the per-pixel "over" of
their renders (Alg. 1).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import core as OC


def render_multi(scenes: Sequence, insts: Sequence[Optional[OC.Instance]], ray_o, ray_d, t_scalar: float,
                 t_stop: float, dtypes_round=None, density: str = "softplus"):
    """scenes: objects with depth, leaf_ijk, hh, wsig, basis, gamma (and optionally the rounded payload via
    dtypes_round: a function scene -> (hh, wsig)); returns rgb [n,3], alpha, depth, nsamp, margin [n]
    (smallest relative distance of T to t_stop at a stop test) and min_piece [n] (shortest composited
    piece, in leaf units of the finest instance). density: the activation of Eq. 5 ("softplus" or
    "relu")."""
    o = np.asarray(ray_o, np.float32)
    d = np.asarray(ray_d, np.float32)
    n = o.shape[0]
    per = []
    for sc, inst in zip(scenes, insts):
        hh, ws = (sc.hh, sc.wsig) if dtypes_round is None else dtypes_round(sc)
        r = OC.render(sc.depth, sc.leaf_ijk, hh, ws, sc.basis, sc.gamma, o, d, None, t_scalar, 0.0, inst,
                      segments=True, density=density)
        per.append(r)
    dw = np.linalg.norm(d.astype(np.float64), axis=1)
    out = dict(rgb=np.zeros((n, 3)), alpha=np.zeros(n), depth=np.full(n, np.inf), nsamp=np.zeros(n, np.int32),
               margin=np.full(n, np.inf), min_piece=np.full(n, np.inf))
    for r in range(n):
        segs: List[np.ndarray] = []
        for k, res in enumerate(per):
            m = int(res["nsamp"][r])
            if m:
                s = res["seg"][r, :m].copy()
                s[:, 2] *= res["len"][r]                       # kappa: extinction per unit u
                segs.append(s)
        if not segs:
            continue
        allseg = np.concatenate(segs)
        bounds = np.unique(np.concatenate([allseg[:, 0], allseg[:, 1]]))
        T = 1.0
        col = np.zeros(3)
        wsum = dsum = 0.0
        ns = 0
        for a, b in zip(bounds[:-1], bounds[1:]):
            act = allseg[(allseg[:, 0] <= a) & (allseg[:, 1] >= b)]
            if act.shape[0] == 0:
                continue
            kap = act[:, 2]
            ksum = kap.sum()
            lens = [per[k]["len"][r] for k in range(len(per)) if per[k]["nsamp"][r]]
            out["min_piece"][r] = min(out["min_piece"][r], (b - a) * max(lens))
            c = (kap[:, None] * act[:, 3:6]).sum(0) / ksum
            tau = ksum * (b - a)
            alpha = -np.expm1(-tau)
            w = T * alpha
            col += w * c
            wsum += w
            dsum += w * 0.5 * (a + b) * dw[r]
            T *= np.exp(-tau)
            ns += 1
            if t_stop > 0.0:
                out["margin"][r] = min(out["margin"][r], abs(T - t_stop) / t_stop)
                if T < t_stop:
                    break
        out["rgb"][r] = col
        out["alpha"][r] = wsum
        out["depth"][r] = dsum / wsum if wsum > 0 else np.inf
        out["nsamp"][r] = ns
    return out
