"""GPU parity of the spotlight shadow and falloff (Sec. 5.2 "Spotlight
Lighting") against the FP64 lighting oracle: the Gaussian low-pass, the
shading kernel on identical inputs, and the whole chain (the light's alpha map
rendered, low-passed, projected onto the ground; the falloff from the viewer's
depth map) against the oracle's own chain."""
import math

import numpy as np
import pytest

from gpu_util import announce, oracle_render, tdev, upload
from oracle import core as OC
from oracle import lighting as OL
from paper_2202_06088_amd import _lib, ops
from workloads import look_at, orbit_camera, scene_for_workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W,sigma", [(64, 64, 1.5), (37, 129, 2.5), (1, 50, 1.0), (200, 3, 4.0), (96, 96, 16.0)])
def test_blur_matches_oracle(H, W, sigma):
    rng = np.random.default_rng(H * 1000 + W)
    img = rng.random((H, W)).astype(np.float32)
    img[img < 0.6] = 0.0                       # alpha-map-like: flat regions and edges
    announce(f"blur {H}x{W} sigma={sigma}")
    gpu = ops.blur(tdev(img), sigma).cpu().numpy().astype(np.float64)
    ref = OL.blur(img, sigma)
    assert np.abs(gpu - ref).max() <= 2e-6, np.abs(gpu - ref).max()


def make_light(sc, W=128, H=96, k=0.75, r0=0.0):
    """A point light above and beside the leaves' centroid, looking at it; the ground is the
    plane under the lowest leaf."""
    cen = sc.leaf_ijk.mean(0) + 0.5
    G = sc.G
    pos = cen + np.array([0.35 * G, -0.25 * G, 0.9 * G])
    c2w = look_at(pos, cen)
    f = 0.5 * W / math.tan(math.radians(35.0))
    ol = OL.Light(W, H, (f, f, W / 2, H / 2), np.asarray(c2w, np.float32), float(sc.leaf_ijk[:, 2].min()),
                  (0.7, 0.65, 0.6), (0.05, 0.1, 0.2), k, r0)
    cs = _lib.make_camera(W, H, f, f, W / 2, H / 2, np.asarray(c2w, np.float32))
    gl = _lib.make_light(cs, ol.ground_z, ol.ground_rgb, ol.background_rgb, k, r0)
    return ol, gl


def viewer_rays(sc, W=96, H=72):
    cen = sc.leaf_ijk.mean(0) + 0.5
    cam = orbit_camera(cen, 2.2 * sc.G, 0.7, math.radians(25.0), W, H, 45.0)
    o, d = OC.pinhole_rays(W, H, cam.intr(), cam.c2w)
    return o, d


@pytest.mark.parametrize("k,r0", [(0.75, 0.0), (1.0, 40.0), (0.0, 25.0)])
def test_shade_kernel_on_identical_inputs(k, r0):
    """Oracle-made maps fed to both sides: isolates the shading arithmetic."""
    sc = scene_for_workload("tiny")
    ol, gl = make_light(sc, k=k, r0=r0)
    lo, ld = OC.pinhole_rays(ol.width, ol.height, ol.intr, ol.c2w)
    lmap = oracle_render(sc, lo, ld, None, 3.0, 1e-4)["alpha"].reshape(ol.height, ol.width)
    smap = OL.blur(lmap, 1.5).astype(np.float32)
    o, d = viewer_rays(sc)
    v = oracle_render(sc, o, d, None, 3.0, 1e-4)
    rgb, alpha, depth = v["rgb"].astype(np.float32), v["alpha"].astype(np.float32), v["depth"].astype(np.float32)
    announce(f"shade kernel k={k} r0={r0}: {int((alpha > 0).sum())} performer pixels")
    ref = OL.shade(ol, smap, o, d, rgb, alpha, depth)
    gpu = ops.shade(gl, tdev(smap), tdev(o), tdev(d), tdev(rgb), tdev(alpha), tdev(depth)).cpu().numpy()
    err = np.abs(gpu - ref).max()
    announce(f"shade kernel max-abs {err:.2e}; shadowed ground pixels {int((ref < 0.99 * np.asarray(ol.ground_rgb)).all(1).sum())}")
    assert err <= 2e-5, err
    # without a shadow map: plain ground
    ref0 = OL.shade(ol, None, o, d, rgb, alpha, depth)
    gpu0 = ops.shade(gl, None, tdev(o), tdev(d), tdev(rgb), tdev(alpha), tdev(depth)).cpu().numpy()
    assert np.abs(gpu0 - ref0).max() <= 2e-5


def test_shadow_and_falloff_chain():
    """The whole effect: the light's alpha map rendered and low-passed, the viewer image
    rendered with depth, then shaded; GPU chain against the oracle's chain."""
    sc = scene_for_workload("tiny")
    tree = upload(sc)
    ol, gl = make_light(sc, k=0.8, r0=30.0)
    announce("lighting chain: light map render + blur + viewer render + shade")
    lo, ld = OC.pinhole_rays(ol.width, ol.height, ol.intr, ol.c2w)
    ref_map = OL.blur(oracle_render(sc, lo, ld, None, 3.0, 1e-4)["alpha"].reshape(ol.height, ol.width), 1.5)
    o, d = viewer_rays(sc)
    v = oracle_render(sc, o, d, None, 3.0, 1e-4)
    ref = OL.shade(ol, ref_map, o, d, v["rgb"], v["alpha"], v["depth"])
    lrays = ops.pinhole_rays(gl.camera)
    _, la, _, _ = ops.render(tree, lrays[0], lrays[1], 3.0, None, 1e-4, ol.width)
    smap = ops.blur(la.view(ol.height, ol.width), 1.5)
    oo, dd = tdev(o), tdev(d)
    rgb, alpha, depth, _ = ops.render(tree, oo, dd, 3.0, None, 1e-4, 96)
    gpu = ops.shade(gl, smap, oo, dd, rgb, alpha, depth).cpu().numpy()
    err = np.abs(gpu - ref).max()
    sh = (ref < 0.95 * np.asarray(ol.ground_rgb)).all(1) & (v["alpha"] == 0)
    announce(f"lighting chain max-abs {err:.2e}; shadowed ground pixels {int(sh.sum())}")
    assert sh.sum() > 50
    assert err <= 2e-5, err


def test_light_map_on_a_second_stream():
    """The lit frame as the benchmark times it: the light map and its low-pass on a second
    stream while the viewer render runs, the shading waiting for both. Bit-identical to the
    same calls made one after the other."""
    import torch
    sc = scene_for_workload("tiny")
    tree = upload(sc)
    ol, gl = make_light(sc, k=0.8, r0=30.0)
    lo, ld = ops.pinhole_rays(gl.camera)
    o, d = viewer_rays(sc)
    oo, dd = tdev(o), tdev(d)
    announce("lighting chain with the light map on a second stream")
    _, la, _, _ = ops.render(tree, lo, ld, 3.0, None, 1e-4, ol.width)
    ref_map = ops.blur(la.view(ol.height, ol.width), 1.5)
    rgb, alpha, depth, ns = ops.render(tree, oo, dd, 3.0, None, 1e-4, 96)
    ref = ops.shade(gl, ref_map, oo, dd, rgb, alpha, depth)
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    la2 = torch.full_like(la, -1.0)
    lrgb2 = torch.empty(la.shape[0], 3, device=la.device)
    lns2 = torch.empty(la.shape[0], dtype=torch.int32, device=la.device)
    smap2 = torch.full_like(ref_map, -1.0)
    rgb2, alpha2, depth2 = torch.full_like(rgb, -1.0), torch.full_like(alpha, -1.0), torch.full_like(depth, -1.0)
    ns2 = torch.full_like(ns, -1)
    out2 = torch.full_like(ref, -1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        go, ready = torch.cuda.Event(), torch.cuda.Event()
        go.record(main)
        side.wait_event(go)
        _lib.neuvv_render(tree.struct(), None, la.shape[0], lo, ld, None, 3.0, ol.width, 1e-4, lrgb2, la2, None,
                          lns2, side)
        _lib.neuvv_blur(ol.height, ol.width, la2, 1.5, smap2, side)
        ready.record(side)
        _lib.neuvv_render(tree.struct(), None, oo.shape[0], oo, dd, None, 3.0, 96, 1e-4, rgb2, alpha2, depth2, ns2,
                          main)
        main.wait_event(ready)
        _lib.neuvv_shade(gl, smap2, oo.shape[0], oo, dd, rgb2, alpha2, depth2, out2, main)
        torch.cuda.synchronize()
        assert torch.equal(smap2, ref_map)
        assert torch.equal(rgb2, rgb) and torch.equal(alpha2, alpha) and torch.equal(ns2, ns)
        assert torch.equal(out2, ref)
