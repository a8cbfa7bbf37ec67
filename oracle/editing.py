"""Oracle of appearance editing (Sec. 5.2 "Appearance editing").

TEST INFRASTRUCTURE ONLY: used by tests/; the product never imports it.

Readings of the paper's description:
* Each leaf carries 5 more channels: a target colour c_d (3), a target
  density sigma_d (used when >= 0, else the leaf keeps its own density) and a
  first frame t_d; the edit is active at local times tau >= t_d (t_d = +inf:
  never). The renderer then uses c_d (and sigma_d) for that leaf's samples
  (``oracle.core.render(..., edit=...)``).
* Painting a 2-D pattern from a camera: each pixel's ray is traced and the
  terminating voxel is the leaf of the first sample after which the
  accumulated alpha exceeds the threshold (0.99 in the paper), i.e. the leaf
  where the ray stops with t_stop = 1 - threshold (``last_leaf`` of
  ``oracle.core.render``). Rays that never pass the threshold paint nothing.
  When several rays end in the same leaf, the lowest ray index wins.
"""
from __future__ import annotations

import numpy as np


def empty_edits(n_leaves: int) -> np.ndarray:
    """Edit table [N, 5] with every edit inactive (t_d = +inf)."""
    e = np.zeros((n_leaves, 5))
    e[:, 3] = -1.0
    e[:, 4] = np.inf
    return e


def paint(edit: np.ndarray, last_leaf: np.ndarray, colours: np.ndarray, sigma_d: float, t_d: float) -> np.ndarray:
    """Returns a copy of the edit table [N, 5] with the leaves hit by the rays set to
    (colour of the lowest-index ray ending there, sigma_d, t_d)."""
    out = np.array(edit, np.float64, copy=True)
    last_leaf = np.asarray(last_leaf, np.int64)
    colours = np.asarray(colours, np.float64).reshape(-1, 3)
    rays = np.nonzero(last_leaf >= 0)[0]
    winner = {}
    for r in rays:                       # ascending ray index: the first seen wins
        winner.setdefault(int(last_leaf[r]), int(r))
    for leaf, r in winner.items():
        out[leaf, :3] = colours[r]
        out[leaf, 3] = sigma_d
        out[leaf, 4] = t_d
    return out
