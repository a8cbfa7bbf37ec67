"""GPU parity of the exact per-ray merge of placed instances (up to 4,
interpenetrating, duplicated, different trees, 16-bit storage) against the
merge oracle, which is itself pinned against the single render, Alg. 1 and
closed forms."""
import math

import numpy as np
import pytest
import torch

from gpu_util import announce, compare, tiny_camera, inst_pair, round_storage, tdev, upload
from oracle import core as OC
from oracle import multi as OM
from paper_2202_06088_amd import _lib
from workloads import make_scene, random_rays, scene_for_workload

pytestmark = pytest.mark.gpu


def rot_z(th):
    return np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], np.float32)


def around_centre(sc, th, shift, scale=1.0, off=0.0, wrap=0):
    """Instance rotating the tree by th about the vertical axis through its leaves' centroid, then shifting."""
    c = sc.leaf_ijk.mean(0) + 0.5
    R = rot_z(th)
    trans = (c - scale * (R @ c) + np.asarray(shift)).astype(np.float32)
    return inst_pair(R, trans, scale, off, wrap)


def gpu_multi(trees, ginsts, o, d, t, t_stop, image_width=0):
    n = o.shape[0]
    rgb = torch.empty(n, 3, device="cuda")
    alpha = torch.empty(n, device="cuda")
    depth = torch.empty(n, device="cuda")
    nsamp = torch.empty(n, dtype=torch.int32, device="cuda")
    _lib.neuvv_render_multi([tr.struct() for tr in trees], ginsts, n, tdev(o), tdev(d), None, t, image_width, t_stop,
                            rgb, alpha, depth, nsamp)
    torch.cuda.synchronize()
    return dict(rgb=rgb.cpu().numpy().astype(np.float64), alpha=alpha.cpu().numpy().astype(np.float64),
                depth=depth.cpu().numpy().astype(np.float64), nsamp=nsamp.cpu().numpy())


def ref_multi(scenes, oinsts, o, d, t, t_stop, dtype=_lib.F32):
    rnd = None
    if dtype != _lib.F32:
        def rnd(sc):
            return round_storage(sc.hh, dtype), round_storage(sc.wsig, dtype)
    r = OM.render_multi(scenes, oinsts, o, d, t, t_stop, dtypes_round=rnd)
    r["margin"] = np.stack([r["min_piece"], r["margin"]], 1)
    return r


@pytest.fixture(scope="module")
def scenes():
    announce("multi: two scenes (tiny workload and a depth-6 humanoid)")
    return scene_for_workload("tiny"), make_scene(6, 15_000, "human", seed=71, T=30)


def test_single_instance_equals_render(scenes):
    sc = scenes[0]
    tree = upload(sc)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    oi, gi = around_centre(sc, 0.3, [1.0, -0.5, 0.25], 1.1, 2.5, 1)
    announce("multi L=1")
    ref = ref_multi([sc], [oi], o, d, 3.0, 1e-4)
    gpu = gpu_multi([tree], [gi], o, d, 3.0, 1e-4, 64)
    compare(gpu, ref, label="multi L=1")


@pytest.mark.parametrize("t_stop", [0.0, 1e-4])
def test_two_interpenetrating_instances(scenes, t_stop):
    sc = scenes[0]
    tree = upload(sc)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    a = around_centre(sc, 0.0, [0.0, 0.0, 0.0])
    b = around_centre(sc, 0.8, [2.0, 1.0, -1.0], 0.9, 7.0, 1)
    announce(f"multi L=2 interpenetrating t_stop={t_stop}")
    ref = ref_multi([sc, sc], [a[0], b[0]], o, d, 4.0, t_stop)
    gpu = gpu_multi([tree, tree], [a[1], b[1]], o, d, 4.0, t_stop, 64)
    st = compare(gpu, ref, label=f"multi L=2 t_stop={t_stop}")
    single = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 4.0, t_stop, a[0])
    assert (ref["nsamp"] > single["nsamp"]).sum() > 100            # the instances really overlap
    assert st["hit"] > 500


def test_four_instances_two_trees_duplicates_and_random_rays(scenes):
    s1, s2 = scenes
    t1, t2 = upload(s1), upload(s2)
    insts = [around_centre(s1, 0.0, [0, 0, 0]), around_centre(s1, 0.0, [0, 0, 0]),       # a duplicate
             around_centre(s2, 1.2, [3.0, -2.0, 0.0], 1.0, 5.0, 1), around_centre(s2, -0.7, [-4.0, 2.0, 1.0], 1.3)]
    rng = np.random.default_rng(72)
    o, d = random_rays(64, 3000, rng, inside_frac=0.2)
    announce("multi L=4 (duplicate + two placements of a second tree), random rays")
    ref = ref_multi([s1, s1, s2, s2], [x[0] for x in insts], o, d, 6.5, 1e-4)
    gpu = gpu_multi([t1, t1, t2, t2], [x[1] for x in insts], o, d, 6.5, 1e-4)
    compare(gpu, ref, label="multi L=4")


@pytest.mark.parametrize("dtype", [_lib.F16, _lib.BF16])
def test_multi_16bit(scenes, dtype):
    sc = scenes[1]
    tree = upload(sc, dtype)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    a = around_centre(sc, 0.0, [0, 0, 0])
    b = around_centre(sc, 0.5, [1.5, 0.0, 0.0], 1.0, 3.0, 0)
    announce(f"multi L=3 storage {dtype}")
    ref = ref_multi([sc, sc, sc], [a[0], b[0], a[0]], o, d, 2.0, 1e-4, dtype)
    gpu = gpu_multi([tree, tree, tree], [a[1], b[1], a[1]], o, d, 2.0, 1e-4, 64)
    compare(gpu, ref, label=f"multi dtype={dtype}")


def test_lists_and_fused_fallback_agree(scenes):
    """The two-phase merge gives every ray 2 list entries per instance of room; rays whose
    lists do not fit are rendered by the fused kernel instead. Rays with at least 8 composited
    intervals, rendered alone, cannot all fit (each composited interval ends at a list entry of
    some instance), so part of them take the fused kernel; rendered among 100x as many rays that
    miss every instance, their lists fit. Both calls must agree, and match the oracle."""
    sc = scenes[0]
    tree = upload(sc)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    a = around_centre(sc, 0.0, [0.0, 0.0, 0.0])
    b = around_centre(sc, 0.8, [2.0, 1.0, -1.0], 0.9, 7.0, 1)
    first = gpu_multi([tree, tree], [a[1], b[1]], o, d, 4.0, 1e-4)
    keep = first["nsamp"] >= 8
    o, d = o[keep], d[keep]
    n = o.shape[0]
    assert n >= 200, n
    announce(f"multi L=2: {n} rays alone and among {100 * n} missing rays")
    alone = gpu_multi([tree, tree], [a[1], b[1]], o, d, 4.0, 1e-4)
    assert alone["nsamp"].sum() > 2 * 2 * n            # more intervals than the room of the call holds
    om = np.tile(np.array([[-1.0e4, -1.0e4, -1.0e4]], np.float32), (100 * n, 1))
    dm = np.tile(np.array([[-1.0, 0.25, 0.0]], np.float32), (100 * n, 1))
    among = gpu_multi([tree, tree], [a[1], b[1]], np.concatenate([o, om]), np.concatenate([d, dm]), 4.0, 1e-4)
    assert np.all(among["nsamp"][n:] == 0) and np.all(among["alpha"][n:] == 0.0)
    for k in ("rgb", "alpha", "depth", "nsamp"):
        x, y = alone[k], among[k][:n]
        fin = np.isfinite(y)
        assert np.array_equal(np.isfinite(x), fin), k
        err = np.abs(x[fin] - y[fin]).max() if fin.any() else 0.0
        announce(f"alone vs among, {k}: max-abs {err:.2e}")
        assert err <= (0 if k == "nsamp" else 1e-6 * max(1.0, np.abs(y[fin]).max())), (k, err)
    ref = ref_multi([sc, sc], [a[0], b[0]], o, d, 4.0, 1e-4)
    compare(alone, ref, label="multi L=2 rays alone")
    compare({k: v[:n] for k, v in among.items()}, ref, label="multi L=2 rays among missing rays")


def test_multi_per_ray_time(scenes):
    """Rays with their own time: each ray takes one of three times, and every group matches the
    merge oracle run with that time for all its rays."""
    sc = scenes[0]
    tree = upload(sc)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    a = around_centre(sc, 0.0, [0.0, 0.0, 0.0], 1.0, 0.0, 1)
    b = around_centre(sc, 0.8, [2.0, 1.0, -1.0], 0.9, 7.0, 1)
    times = np.array([0.0, 4.25, 17.5], np.float32)
    which = np.arange(o.shape[0]) % 3
    t = times[which]
    n = o.shape[0]
    announce("multi L=2 with per-ray times")
    rgb = torch.empty(n, 3, device="cuda")
    alpha = torch.empty(n, device="cuda")
    depth = torch.empty(n, device="cuda")
    nsamp = torch.empty(n, dtype=torch.int32, device="cuda")
    _lib.neuvv_render_multi([tree.struct(), tree.struct()], [a[1], b[1]], n, tdev(o), tdev(d), tdev(t), 0.0, 0,
                            1e-4, rgb, alpha, depth, nsamp)
    torch.cuda.synchronize()
    gpu = dict(rgb=rgb.cpu().numpy().astype(np.float64), alpha=alpha.cpu().numpy().astype(np.float64),
               depth=depth.cpu().numpy().astype(np.float64), nsamp=nsamp.cpu().numpy())
    for k, tk in enumerate(times):
        m = which == k
        ref = ref_multi([sc, sc], [a[0], b[0]], o[m], d[m], float(tk), 1e-4)
        compare({key: v[m] for key, v in gpu.items()}, ref, label=f"multi per-ray t = {tk}")
