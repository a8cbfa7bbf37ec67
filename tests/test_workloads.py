"""Seeded workload generators: determinism, target leaf counts, camera framing."""
import numpy as np

from workloads import WORKLOADS, make_scene, ring_cameras, scene_for_workload


def test_seeded_and_deterministic():
    a = make_scene(6, 20_000, "random", seed=1, T=30)
    b = make_scene(6, 20_000, "random", seed=1, T=30)
    for k in ("leaf_ijk", "hh", "wsig", "basis", "gamma"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = make_scene(6, 20_000, "random", seed=2, T=30)
    assert not np.array_equal(a.hh[:10], c.hh[:10])


def test_tiny_and_reduced_humanoid_counts():
    s1 = scene_for_workload("tiny")
    assert abs(s1.n_leaves - 20_000) <= 0.02 * 20_000
    assert s1.hh.shape == (s1.n_leaves, 3, 16) and s1.wsig.shape == (s1.n_leaves, 8)
    assert s1.basis.shape == (30, 8) and s1.gamma.shape == (30,)
    assert np.all(s1.leaf_ijk >= 0) and np.all(s1.leaf_ijk < 64)
    keys = s1.leaf_ijk[:, 0] + 64 * (s1.leaf_ijk[:, 1] + 64 * s1.leaf_ijk[:, 2].astype(np.int64))
    assert np.all(np.diff(keys) > 0)          # sorted, no duplicates
    h = make_scene(7, 30_000, "human", seed=2)
    assert abs(h.n_leaves - 30_000) <= 0.02 * 30_000
    assert h.n_leaves / 128 ** 3 < 0.05        # a few per cent of the cube


def test_ring_cameras_look_at_blob():
    s = make_scene(6, 8000, "human", seed=3)
    cams = ring_cameras(s, 8, 64, 36, 40.0, 10.0, seed=4)
    ctr = (s.leaf_ijk.min(0) + s.leaf_ijk.max(0) + 1) / 2.0
    for c in cams:
        eye = c.c2w[:, 3].astype(np.float64)
        fwd = c.c2w[:, 2].astype(np.float64)
        v = ctr - eye
        assert np.dot(v / np.linalg.norm(v), fwd) > 0.999
    assert set(WORKLOADS) == {"tiny", "forward", "train", "mixed", "multi"}
