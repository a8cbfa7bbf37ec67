"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: FP32 forward max|gpu - oracle| <= 1e-5 max|oracle| (rgb, alpha,
depth), sample counts identical except where the oracle reports an
ambiguous stop or a sub-1e-5 segment; gradients <= 1e-4 relative to the
largest entry; 16-bit storage compared on the rounded payload to the same
1e-5, and against the unrounded payload to 2e-3 max-abs for FP16.
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import (DEV, announce, cam_struct, compare, tiny_camera, gpu_render, inst_pair, oracle_render,
                      rel_err, round_storage, tdev, upload)
from oracle import core as OC
from oracle.hh import hh_basis
from paper_2202_06088_amd import _lib, ops
from workloads import make_scene, random_rays, scene_for_workload, special_rays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny_scene():
    return scene_for_workload("tiny")


@pytest.fixture(scope="module")
def tiny_tree(tiny_scene):
    return upload(tiny_scene)


def test_eval_hh_matches_oracle():
    announce("eval_hh K=30, 4096 random directions")
    rng = np.random.default_rng(0)
    d = rng.normal(size=(4096, 3)).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.uniform(0, math.pi, 4096).astype(np.float32)
    out = ops.eval_hh(30, tdev(d), tdev(g)).cpu().numpy()
    ref = hh_basis(30, d.astype(np.float64), g.astype(np.float64))
    assert np.abs(out - ref).max() < 2e-6
    out16 = ops.eval_hh(16, tdev(d), tdev(g)).cpu().numpy()
    assert np.array_equal(out16, out[:, :16])


def test_pinhole_matches_oracle():
    from workloads import orbit_camera
    for (W, H) in ((64, 64), (67, 45), (1920, 1080)):
        cam = orbit_camera((300.0, 250.0, 200.0), 1400.0, 0.9, 0.17, W, H, 40.0)
        announce(f"pinhole {W}x{H}")
        o, d = ops.pinhole_rays(cam_struct(cam))
        ro, rd = OC.pinhole_rays(W, H, cam.intr(), cam.c2w)
        o, d = o.cpu().numpy(), d.cpu().numpy()
        assert np.array_equal(o, ro)
        diff = d.view(np.int32).astype(np.int64) - rd.view(np.int32).astype(np.int64)
        assert np.abs(diff).max() <= 1
        assert (diff != 0).sum() <= max(1, 1e-6 * diff.size), int((diff != 0).sum())
    pix = torch.tensor([0, 5, 1919, 1920 * 1079 + 7], dtype=torch.int32, device=DEV)
    o2, d2 = ops.pinhole_rays(cam_struct(cam), pix)
    assert np.array_equal(d2.cpu().numpy(), d[pix.cpu().numpy()])


@pytest.mark.parametrize("t_stop", [0.0, 1e-4])
def test_render_tiny_fp32(tiny_scene, tiny_tree, t_stop):
    """Tiny VOctree: depth 6, ~20k leaves, 64x64 pinhole view, one seeded frame."""
    cam = tiny_camera(tiny_scene)
    t = float(np.random.default_rng(12).integers(0, tiny_scene.T))
    announce(f"tiny render t_stop={t_stop} t={t}")
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    go, gd = ops.pinhole_rays(cam_struct(cam))
    assert np.array_equal(go.cpu().numpy(), o) and np.array_equal(gd.cpu().numpy(), d)
    ref = oracle_render(tiny_scene, o, d, None, t, t_stop)
    # rays as a row-major 64-wide image (8x8 tiles per wavefront) and as a flat list
    for iw in (64, 0):
        rgb, alpha, depth, nsamp = ops.render(tiny_tree, go, gd, t, None, t_stop, iw)
        torch.cuda.synchronize()
        gpu = dict(rgb=rgb.cpu().numpy().astype(np.float64), alpha=alpha.cpu().numpy().astype(np.float64),
                   depth=depth.cpu().numpy().astype(np.float64), nsamp=nsamp.cpu().numpy())
        st = compare(gpu, ref, label=f"tiny_scene iw={iw}")
        assert st["hit"] > 500


@pytest.mark.parametrize("depth,n_leaves,seed", [(2, 30, 0), (4, 1500, 1), (6, 30000, 2)])
def test_render_random_and_special_rays(depth, n_leaves, seed):
    sc = make_scene(depth, n_leaves, "random", seed=seed, T=7)
    tree = upload(sc)
    rng = np.random.default_rng(100 + seed)
    o1, d1 = random_rays(sc.G, 3000, rng, inside_frac=0.2)
    o2, d2 = special_rays(sc.G)
    o = np.concatenate([o1, o2])
    d = np.concatenate([d1, d2])
    t = rng.uniform(0, sc.T, o.shape[0]).astype(np.float32)
    for t_stop in (0.0, 1e-2):
        announce(f"random rays depth={depth} t_stop={t_stop}")
        ref = oracle_render(sc, o, d, t, 0.0, t_stop)
        gpu = gpu_render(tree, o, d, t, 0.0, t_stop)
        compare(gpu, ref, label=f"random d={depth}")


def test_render_edge_cases():
    # empty tree: every ray misses
    sc = make_scene(4, 100, "random", seed=3, T=5)
    o, d = random_rays(16, 500, np.random.default_rng(1))
    empty = type(sc)(4, np.zeros((0, 3), np.int32), np.zeros((0, 3, 16), np.float32), np.zeros((0, 8), np.float32),
                     sc.basis, sc.gamma)
    announce("edge: empty tree")
    g = gpu_render(upload(empty), o, d, None, 1.0)
    assert np.all(g["rgb"] == 0) and np.all(g["alpha"] == 0) and np.all(g["nsamp"] == 0)
    assert np.all(np.isinf(g["depth"]))
    # zero rays
    announce("edge: zero rays")
    tree = upload(sc)
    z = torch.zeros(0, 3, device=DEV)
    out = ops.render(tree, z, z, 0.0)
    assert out[0].shape == (0, 3)
    # ragged image: 67 x 45 rays with the 8x8 tile mapping
    announce("edge: ragged 67x45 image tiles")
    rng = np.random.default_rng(5)
    o, d = random_rays(16, 67 * 45, rng)
    ref = oracle_render(sc, o, d, None, 2.0, 1e-4)
    gpu = gpu_render(tree, o, d, None, 2.0, 1e-4, image_width=67)
    compare(gpu, ref, label="ragged")
    # non-multiple of the width: the last row is partial
    gpu = gpu_render(tree, o[:67 * 44 + 13], d[:67 * 44 + 13], None, 2.0, 1e-4, image_width=67)
    for k in ("rgb", "alpha", "nsamp"):
        assert np.array_equal(gpu[k], gpu_render(tree, o, d, None, 2.0, 1e-4)[k][:67 * 44 + 13])
    # depth 1 and depth 12 (maximum) trees
    r = np.random.default_rng(9)
    ijk1 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 1], [0, 1, 1], [0, 0, 1]], np.int32)
    # depth 12: a dense 12^3 cluster near the centre plus 300 cells scattered over the 4096^3 grid
    cl = np.stack(np.meshgrid(*[np.arange(2040, 2052)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sc_ = r.integers(0, 4096, (300, 3))
    ijk12 = np.unique(np.concatenate([cl, sc_]), axis=0).astype(np.int32)
    for depth, ijk in ((1, ijk1), (12, ijk12)):
        announce(f"edge: depth {depth}")
        n = ijk.shape[0]
        s2 = type(sc)(depth, ijk, r.normal(0, 0.3, (n, 3, 16)).astype(np.float32),
                      r.normal(size=(n, 8)).astype(np.float32), sc.basis, sc.gamma)
        if depth == 12:
            v = r.normal(size=(2000, 3))
            v /= np.linalg.norm(v, axis=1, keepdims=True)
            o = (2046.0 + 40.0 * v).astype(np.float32)
            d = (2046.0 + r.uniform(-8, 8, (2000, 3)) - o).astype(np.float32)
            o2, d2 = random_rays(s2.G, 500, r)
            o, d = np.concatenate([o, o2]), np.concatenate([d, d2])
        else:
            o, d = random_rays(s2.G, 2000, np.random.default_rng(depth))
        ref = oracle_render(s2, o, d, None, 1.5, 1e-4)
        gpu = gpu_render(upload(s2), o, d, None, 1.5, 1e-4)
        compare(gpu, ref, label=f"depth{depth}")


@pytest.mark.parametrize("dtype", [_lib.F16, _lib.BF16])
def test_render_16bit_storage(tiny_scene, dtype):
    cam = tiny_camera(tiny_scene)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    tree = upload(tiny_scene, dtype)
    announce(f"16-bit storage dtype={dtype}")
    gpu = gpu_render(tree, o, d, None, 3.0, 1e-4)
    ref_r = oracle_render(tiny_scene, o, d, None, 3.0, 1e-4, dtype=dtype)
    compare(gpu, ref_r, label=f"dtype{dtype} vs rounded payload")
    ref = oracle_render(tiny_scene, o, d, None, 3.0, 1e-4)
    err = np.abs(gpu["rgb"] - ref["rgb"]).max()
    mse = np.mean((gpu["rgb"] - ref["rgb"]) ** 2)
    psnr = 10 * math.log10(1.0 / mse) if mse > 0 else math.inf
    announce(f"dtype {dtype}: max-abs {err:.3e}, PSNR {psnr:.1f} dB vs FP64 on unrounded payload")
    if dtype == _lib.F16:
        assert err <= 2e-3
    assert psnr > 40


def test_instances_match_oracle():
    sc = make_scene(5, 4000, "human", seed=21, T=40)
    tree = upload(sc)
    rng = np.random.default_rng(22)
    G = sc.G
    th = 1.1
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], np.float32)
    s = 1.7
    trans = np.array([10.0, -20.0, 3.0], np.float32)
    centre = s * (R.astype(np.float64) @ np.full(3, G / 2.0)) + trans
    v = rng.normal(size=(2500, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o = (centre + 2.2 * s * G * v).astype(np.float32)
    tgt = centre + rng.uniform(-0.5, 0.5, (2500, 3)) * s * G
    d = (tgt - o).astype(np.float32)
    for off, wrap, t in ((0.0, False, 5.5), (33.25, True, 20.0), (-7.5, True, 3.0), (50.0, False, 1.0)):
        oi, gi = inst_pair(R, trans, s, off, wrap)
        announce(f"instance off={off} wrap={wrap} t={t}")
        ref = oracle_render(sc, o, d, None, t, 1e-4, inst=oi)
        gpu = gpu_render(tree, o, d, None, t, 1e-4, inst=gi)
        st = compare(gpu, ref, label="instance")
        assert st["hit"] > 200


def test_compose_matches_oracle():
    rng = np.random.default_rng(31)
    for L, n in ((1, 100), (2, 5000), (4, 100_003), (16, 2000)):
        announce(f"compose L={L} n={n}")
        P = rng.uniform(0, 0.6, (L, n, 3)).astype(np.float32)
        A = rng.uniform(0, 1, (L, n)).astype(np.float32)
        D = rng.uniform(0, 10, (L, n)).astype(np.float32)
        D[:, : n // 10] = np.round(D[:, : n // 10])          # many exact ties
        D[rng.uniform(size=(L, n)) < 0.1] = np.inf
        gP = rng.normal(size=(n, 3)).astype(np.float32)
        gA = rng.normal(size=n).astype(np.float32)
        o_rgb, o_a, o_d = ops.compose(tdev(P), tdev(A), tdev(D))
        r_rgb, r_a, r_d = OC.compose(P, A, D)
        assert rel_err(o_rgb.cpu().numpy(), r_rgb) < 1e-6
        assert np.abs(o_a.cpu().numpy() - r_a).max() < 1e-6
        assert np.array_equal(o_d.cpu().numpy(), r_d.astype(np.float32))
        g_rgb, g_a = ops.compose_backward(tdev(P), tdev(A), tdev(D), tdev(gP), tdev(gA))
        q_rgb, q_a = OC.compose_grad(P, A, D, gP, gA)
        assert rel_err(g_rgb.cpu().numpy(), q_rgb) < 1e-5
        assert rel_err(g_a.cpu().numpy(), q_a) < 1e-5


@pytest.mark.parametrize("dtype", [_lib.F32, _lib.F16, _lib.BF16])
def test_leaf_rows_layout_same_results(tiny_scene, dtype):
    """The leaf-major payload layout loads the same values: forward outputs are bitwise
    equal to the vector-SoA layout, adjoints equal up to the order of atomic additions."""
    from paper_2202_06088_amd.voctree import VOctree
    cam = tiny_camera(tiny_scene)
    o, d = ops.pinhole_rays(cam_struct(cam))
    trees = [VOctree.build(tiny_scene.depth, tiny_scene.leaf_ijk, tiny_scene.hh, tiny_scene.wsig, tiny_scene.basis, tiny_scene.gamma, dtype, DEV,
                           layout=lay) for lay in (_lib.LAYOUT_VEC_SOA, _lib.LAYOUT_LEAF_ROWS)]
    announce(f"leaf-rows layout, dtype {dtype}")
    outs = [ops.render(tr, o, d, 6.0, None, 1e-4, 64) for tr in trees]
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    g = torch.randn_like(outs[0][0])
    grads = [ops.render_backward(tr, o, d, out[0], out[1], out[3], g, None, 6.0, None, 1e-4, 64)
             for tr, out in zip(trees, outs)]
    torch.cuda.synchronize()
    assert rel_err(grads[1][0].cpu().numpy(), grads[0][0].cpu().numpy()) < 1e-6
    assert rel_err(grads[1][1].cpu().numpy(), grads[0][1].cpu().numpy()) < 1e-6


def _directory_expected(depth, leaf_ijk):
    """The brick directory from its definition, on the occupancy grid alone: per 4^3 region, whether
    it holds a leaf, and for one that holds none the largest s in [2, depth) such that the aligned
    cube of edge 2^s around it holds none."""
    G = 1 << depth
    E = max(G >> 2, 1)
    occ = np.zeros((G, G, G), bool)
    occ[leaf_ijk[:, 2], leaf_ijk[:, 1], leaf_ijk[:, 0]] = True         # [z, y, x]
    reg = occ.reshape(E, G // E, E, G // E, E, G // E).any(axis=(1, 3, 5)).ravel()   # entry (k E + j) E + i
    k, j, i = np.unravel_index(np.arange(E ** 3), (E, E, E))
    s = np.full(E ** 3, 2)
    grow = ~reg
    for lev in range(3, depth):
        f = 1 << (lev - 2)                        # regions per cube edge at this size
        n = E // f
        cube = reg.reshape(n, f, n, f, n, f).any(axis=(1, 3, 5))
        grow &= ~cube[k // f, j // f, i // f]
        s = np.where(grow, lev, s)
    return reg, s, occ


@pytest.mark.parametrize("case", ["d1", "d2", "d3", "tiny", "forward"])
def test_brick_directory_matches_its_definition(case):
    """neuvv_build_directory bit for bit: regions that hold a leaf name their last-level node, whose
    mask is the region's occupancy and whose leaves carry the input cells' slots; the others the
    largest empty aligned cube around them (the walk's skip)."""
    from paper_2202_06088_amd.voctree import build_node_table
    rng = np.random.default_rng(71)
    if case in ("d1", "d2", "d3"):
        depth = int(case[1])
        G = 1 << depth
        cells = np.unique(rng.integers(0, G, (max(G ** 3 // 5, 1), 3)), axis=0).astype(np.int32)
    else:
        sc = scene_for_workload(case)
        depth, cells = sc.depth, sc.leaf_ijk
    nodes, slots = build_node_table(depth, cells)
    n = _lib.neuvv_directory_entries(depth)
    dn = torch.from_numpy(nodes).to(DEV)
    dd = torch.full((n,), 12345, dtype=torch.int32, device=DEV)
    announce(f"directory depth {depth}: {cells.shape[0]} leaves, {n} entries")
    _lib.neuvv_build_directory(depth, nodes.shape[0], dn, dd, n)
    torch.cuda.synchronize()
    got = dd.cpu().numpy()
    if depth <= 2:
        assert np.array_equal(got, np.zeros(1, np.int32))     # the root is the only node
        return
    reg, s, occ = _directory_expected(depth, cells)
    assert np.array_equal(got >= 0, reg)
    assert np.array_equal(-got[~reg] - 1, s[~reg])
    # bricks: mask bit q of the region's cell (x0 | y0<<1 | z0<<2 | x1<<3 | y1<<4 | z1<<5) set exactly
    # where the cell holds a leaf, and that leaf's slot at base + rank
    E = (1 << depth) >> 2
    slot_at = {tuple(c): int(sl) for c, sl in zip(cells.tolist(), slots.tolist())}
    idx = np.nonzero(reg)[0]
    for r in rng.choice(idx, min(idx.size, 3000), replace=False):
        row = nodes[got[r]]
        m = (int(row[1]) & 0xffffffff) << 32 | (int(row[0]) & 0xffffffff)
        bx, by, bz = 4 * (r % E), 4 * ((r // E) % E), 4 * (r // (E * E))
        for q in range(64):
            x = bx + (q & 1) + ((q >> 3) & 1) * 2
            y = by + ((q >> 1) & 1) + ((q >> 4) & 1) * 2
            z = bz + ((q >> 2) & 1) + ((q >> 5) & 1) * 2
            assert bool((m >> q) & 1) == bool(occ[z, y, x])
            if (m >> q) & 1:
                assert int(row[2]) + bin(m & ((1 << q) - 1)).count("1") == slot_at[(x, y, z)]
