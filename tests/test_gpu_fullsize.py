"""Full-size parity in the launch configuration bench.py times: the traced pair
(neuvv_render_trace, then neuvv_render_backward_trace replaying its samples)
with the bench's trace room.

Forward-render workload: depth-9 humanoid VOctree (~2M leaves), 8 cameras at
1920x1080 rendered in one launch (16.6 M rays, 8x8 tiles, t_stop = 1e-4), with
the global hyperangle table (K=16, C=8; and K=30, Table 3's N=30) and with
the paper's per-point leaf (K=14, C=31, Cg=31).
The exact merge of L placements, and the lit frame (the light map on a second
stream, then the shading), run over the same ring as bench.py --multi L and
--lighting time them, and so does appearance editing as --editing runs it (the
terminal leaves of one whole camera, the paint table, the edited ring). Outputs are checked on a seeded sample of pixels that the
FP64 oracle renders one by one. The adjoint is checked in the same launch with the
upstream gradient non-zero only on the sampled pixels, so the oracle's
gradient over those rays is the exact expected result.
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, announce, compare, oracle_render, rel_err, stop_ambiguous, tdev, upload
from oracle import core as OC
from paper_2202_06088_amd import _lib, ops
from workloads import WORKLOADS, make_scene, make_scene_per_point, ring_cameras, scene_for_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["global", "global-k30", "per-point"])
def ring(request):
    announce(f"full size: generating the depth-9 scene ({request.param} hyperangle)")
    if request.param == "global":
        sc = scene_for_workload("forward")
    elif request.param == "global-k30":
        # Table 3's N = 30 (every HH function with n <= 3) on the same occupancy
        c2 = WORKLOADS["forward"]
        sc = make_scene(c2["depth"], c2["target"], c2["kind"], K=30, C=8, T=c2["T"], seed=c2["seed"])
    else:
        c2 = WORKLOADS["forward"]
        sc = make_scene_per_point(c2["depth"], c2["target"], c2["kind"], T=c2["T"], seed=c2["seed"])
    cams = ring_cameras(sc, 8, 1920, 1080, 40.0, 10.0, seed=2)
    t = float(np.random.default_rng(2002).uniform(0, sc.T))
    return sc, cams, t


def test_full_ring_forward_and_adjoint_sampled(ring):
    """The bench's launch configuration (the whole ring in one traced launch, 8x8 tiles),
    both hyperangle forms; parity on sampled rays the oracle renders one by one."""
    sc, cams, t = ring
    W, H = 1920, 1080
    n_cam = W * H
    n = 8 * n_cam
    tree = upload(sc)
    o = torch.empty(n, 3, device=DEV)
    d = torch.empty(n, 3, device=DEV)
    for i, c in enumerate(cams):
        cs = _lib.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.c2w)
        _lib.neuvv_pinhole_rays(cs, n_cam, None, o[i * n_cam:(i + 1) * n_cam], d[i * n_cam:(i + 1) * n_cam])
    announce(f"full size: traced render {n} rays, {sc.n_leaves} leaves")
    # room for one sample per ray, as bench.py gives it (a per-point sample takes two entries)
    trace = ops.Trace(n, n * (2 if tree.Cg > 0 else 1), DEV)
    rgb, alpha, depth, nsamp = ops.render(tree, o, d, t, None, 1e-4, W, trace=trace)
    torch.cuda.synchronize()
    ns = nsamp.cpu().numpy()
    hit = np.nonzero(ns > 0)[0]
    announce(f"full size: {hit.size} hit rays, {int(ns.sum())} samples")
    assert hit.size > 100_000
    rng = np.random.default_rng(77)
    sample = np.unique(np.concatenate([rng.choice(hit, 1500, replace=False), rng.choice(n, 500, replace=False)]))
    cam_idx = sample // n_cam
    pix = (sample % n_cam).astype(np.int32)
    ro = np.zeros((sample.size, 3), np.float32)
    rd = np.zeros((sample.size, 3), np.float32)
    for c in range(8):
        m = cam_idx == c
        if m.any():
            ro[m], rd[m] = OC.pinhole_rays(W, H, cams[c].intr(), cams[c].c2w, pix[m])
    go, gd = o[sample].cpu().numpy(), d[sample].cpu().numpy()
    same = np.all(go == ro, axis=1) & np.all(gd == rd, axis=1)
    assert same.mean() > 0.999, same.mean()
    sample, ro, rd = sample[same], ro[same], rd[same]
    gC = np.random.default_rng(78).normal(size=(sample.size, 3)).astype(np.float32)
    gA = np.random.default_rng(79).normal(size=sample.size).astype(np.float32)
    ref = oracle_render(sc, ro, rd, None, t, 1e-4, g_rgb=gC, g_alpha=gA)
    amb = stop_ambiguous(ref, label="full ring")
    gC[amb] = 0.0
    gA[amb] = 0.0
    ref = oracle_render(sc, ro, rd, None, t, 1e-4, g_rgb=gC, g_alpha=gA)
    sidx = torch.from_numpy(sample).to(DEV)
    gpu = dict(rgb=rgb[sidx].cpu().numpy().astype(np.float64), alpha=alpha[sidx].cpu().numpy().astype(np.float64),
               depth=depth[sidx].cpu().numpy().astype(np.float64), nsamp=nsamp[sidx].cpu().numpy())
    compare(gpu, ref, label="full ring (sampled)")
    # adjoint, same launch configuration, upstream gradient only on the sampled rays
    g_rgb = torch.zeros(n, 3, device=DEV)
    g_alpha = torch.zeros(n, device=DEV)
    g_rgb[sidx] = tdev(gC)
    g_alpha[sidx] = tdev(gA)
    announce("full size: adjoint replayed from the trace")
    out = ops.render_backward(tree, o, d, rgb, alpha, nsamp, g_rgb, g_alpha, t, None, 1e-4, W, trace=trace)
    torch.cuda.synchronize()
    parts = tree.unpack_grad(out[0])
    e = [rel_err(parts[0].cpu().numpy(), ref["grad_hh"]), rel_err(parts[1].cpu().numpy(), ref["grad_wsig"]),
         rel_err(out[1].cpu().numpy(), ref["grad_basis"])]
    if tree.Cg > 0:
        e += [rel_err(parts[2].cpu().numpy(), ref["grad_wgam"]), rel_err(out[2].cpu().numpy(), ref["grad_basis_g"])]
    announce(f"full size adjoint rel errors {e}")
    assert max(e) <= 1e-4


@pytest.mark.parametrize("L", [2, 4])
def test_full_ring_exact_merge_sampled(L):
    """The exact merge as bench.py --multi L times it: L placements of the ring's tree (rotated
    about the vertical axis through the leaves' centroid, shifted, re-timed), the whole ring in
    one launch; parity on sampled rays against the merge oracle."""
    import math
    from oracle import multi as OM
    sc = scene_for_workload("forward")
    cams = ring_cameras(sc, 8, 1920, 1080, 40.0, 10.0, seed=2)
    t = float(np.random.default_rng(2002).uniform(0, sc.T))
    W, H = 1920, 1080
    n_cam = W * H
    n = 8 * n_cam
    tree = upload(sc)
    c = sc.leaf_ijk.mean(0) + 0.5
    g_insts, o_insts = [], []
    for k in range(L):
        th = 2 * math.pi * k / (3 * L)
        R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], np.float32)
        trans = (c - R @ c + np.array([0.04 * sc.G * k, -0.03 * sc.G * k, 0.0])).astype(np.float32)
        g_insts.append(_lib.make_instance(R, trans, 1.0, 37.0 * k, 1))
        o_insts.append(OC.Instance(R, trans, 1.0, 37.0 * k, 1))
    o = torch.empty(n, 3, device=DEV)
    d = torch.empty(n, 3, device=DEV)
    for i, cm in enumerate(cams):
        cs = _lib.make_camera(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.c2w)
        _lib.neuvv_pinhole_rays(cs, n_cam, None, o[i * n_cam:(i + 1) * n_cam], d[i * n_cam:(i + 1) * n_cam])
    rgb = torch.empty(n, 3, device=DEV)
    alpha = torch.empty(n, device=DEV)
    depth = torch.empty(n, device=DEV)
    nsamp = torch.empty(n, dtype=torch.int32, device=DEV)
    announce(f"full size: exact merge of {L} placements over {n} rays")
    _lib.neuvv_render_multi([tree.struct()] * L, g_insts, n, o, d, None, t, W, 1e-4, rgb, alpha, depth, nsamp)
    torch.cuda.synchronize()
    ns = nsamp.cpu().numpy()
    hit = np.nonzero(ns > 0)[0]
    announce(f"full size merge: {hit.size} rays with pieces, {int(ns.sum())} pieces")
    assert hit.size > 100_000
    rng = np.random.default_rng(90 + L)
    sample = np.unique(np.concatenate([rng.choice(hit, 1200, replace=False), rng.choice(n, 300, replace=False)]))
    cam_idx = sample // n_cam
    pix = (sample % n_cam).astype(np.int32)
    ro = np.zeros((sample.size, 3), np.float32)
    rd = np.zeros((sample.size, 3), np.float32)
    for cc in range(8):
        m = cam_idx == cc
        if m.any():
            ro[m], rd[m] = OC.pinhole_rays(W, H, cams[cc].intr(), cams[cc].c2w, pix[m])
    same = np.all(o[sample].cpu().numpy() == ro, axis=1) & np.all(d[sample].cpu().numpy() == rd, axis=1)
    assert same.mean() > 0.999, same.mean()
    sample, ro, rd = sample[same], ro[same], rd[same]
    ref = OM.render_multi([sc] * L, o_insts, ro, rd, t, 1e-4)
    ref["margin"] = np.stack([ref["min_piece"], ref["margin"]], 1)
    idx = torch.from_numpy(sample).to(DEV)
    gpu = dict(rgb=rgb[idx].cpu().numpy().astype(np.float64), alpha=alpha[idx].cpu().numpy().astype(np.float64),
               depth=depth[idx].cpu().numpy().astype(np.float64), nsamp=nsamp[idx].cpu().numpy())
    compare(gpu, ref, label=f"full-size merge L={L}")


def test_full_ring_lit_frame_sampled():
    """The lit frame as bench.py --lighting times it: the light's 256 x 256 alpha map and its
    low-pass on a second stream while the ring renders on the first, then the shading of every
    ring pixel; sampled pixels against the lighting oracle's own chain (its light map rendered
    by the FP64 oracle, low-passed, the viewer pixels rendered by the oracle, shaded)."""
    import math
    from oracle import lighting as OL
    from workloads import look_at
    sc = scene_for_workload("forward")
    cams = ring_cameras(sc, 8, 1920, 1080, 40.0, 10.0, seed=2)
    t = float(np.random.default_rng(2002).uniform(0, sc.T))
    W, H = 1920, 1080
    n_cam = W * H
    n = 8 * n_cam
    tree = upload(sc)
    LW = LH = 256
    cen = sc.leaf_ijk.mean(0) + 0.5
    pos = cen + np.array([0.35 * sc.G, -0.25 * sc.G, 0.9 * sc.G])
    c2w = np.asarray(look_at(pos, cen), np.float32)
    f = 0.5 * LW / math.tan(math.radians(35.0))
    gz = float(sc.leaf_ijk[:, 2].min())
    cam = _lib.make_camera(LW, LH, f, f, LW / 2, LH / 2, c2w)
    light = _lib.make_light(cam, gz, (0.7, 0.65, 0.6), (0.05, 0.1, 0.2), 0.8, 0.5 * sc.G)
    ol = OL.Light(LW, LH, (f, f, LW / 2, LH / 2), c2w, gz, (0.7, 0.65, 0.6), (0.05, 0.1, 0.2), 0.8, 0.5 * sc.G)
    lo, ld = ops.pinhole_rays(cam)
    o = torch.empty(n, 3, device=DEV)
    d = torch.empty(n, 3, device=DEV)
    for i, cm in enumerate(cams):
        cs = _lib.make_camera(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.c2w)
        _lib.neuvv_pinhole_rays(cs, n_cam, None, o[i * n_cam:(i + 1) * n_cam], d[i * n_cam:(i + 1) * n_cam])
    la = torch.empty(LW * LH, device=DEV)
    lrgb = torch.empty(LW * LH, 3, device=DEV)
    lns = torch.empty(LW * LH, dtype=torch.int32, device=DEV)
    smap = torch.empty(LH, LW, device=DEV)
    rgb = torch.empty(n, 3, device=DEV)
    alpha = torch.empty(n, device=DEV)
    depth = torch.empty(n, device=DEV)
    nsamp = torch.empty(n, dtype=torch.int32, device=DEV)
    out = torch.empty(n, 3, device=DEV)
    announce(f"full size: lit frame over {n} rays, light map {LW}x{LH} on a second stream")
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    go, ready = torch.cuda.Event(), torch.cuda.Event()
    go.record(main)
    side.wait_event(go)
    _lib.neuvv_render(tree.struct(), None, LW * LH, lo, ld, None, t, LW, 1e-4, lrgb, la, None, lns, side)
    _lib.neuvv_blur(LH, LW, la, 1.5, smap, side)
    ready.record(side)
    _lib.neuvv_render(tree.struct(), None, n, o, d, None, t, W, 1e-4, rgb, alpha, depth, nsamp, main)
    main.wait_event(ready)
    _lib.neuvv_shade(light, smap, n, o, d, rgb, alpha, depth, out, main)
    torch.cuda.synchronize()
    # the oracle's chain
    lo_h, ld_h = OC.pinhole_rays(LW, LH, ol.intr, ol.c2w)
    lmap = oracle_render(sc, lo_h, ld_h, None, t, 1e-4)["alpha"].reshape(LH, LW)
    smap_ref = OL.blur(lmap, 1.5)
    ns = nsamp.cpu().numpy()
    rng = np.random.default_rng(95)
    hit = np.nonzero(ns > 0)[0]
    sample = np.unique(np.concatenate([rng.choice(hit, 700, replace=False), rng.choice(n, 1300, replace=False)]))
    cam_idx = sample // n_cam
    pix = (sample % n_cam).astype(np.int32)
    ro = np.zeros((sample.size, 3), np.float32)
    rd = np.zeros((sample.size, 3), np.float32)
    for cc in range(8):
        m = cam_idx == cc
        if m.any():
            ro[m], rd[m] = OC.pinhole_rays(W, H, cams[cc].intr(), cams[cc].c2w, pix[m])
    same = np.all(o[sample].cpu().numpy() == ro, axis=1) & np.all(d[sample].cpu().numpy() == rd, axis=1)
    assert same.mean() > 0.999, same.mean()
    sample, ro, rd = sample[same], ro[same], rd[same]
    v = oracle_render(sc, ro, rd, None, t, 1e-4)
    ref = OL.shade(ol, smap_ref, ro, rd, v["rgb"], v["alpha"], v["depth"])
    amb = stop_ambiguous(v, label="lit frame")
    gpu = out[torch.from_numpy(sample).to(DEV)].cpu().numpy().astype(np.float64)
    err = np.abs(gpu - ref)[~amb].max()
    shadowed = ((ref < 0.95 * np.asarray(ol.ground_rgb)).all(1) & (v["alpha"] == 0)).sum()
    announce(f"full-size lit frame: max-abs {err:.2e} over {int((~amb).sum())} pixels, {int(shadowed)} shadowed ground")
    assert shadowed > 20
    assert err <= 2e-5, err


def test_full_ring_editing():
    """Appearance editing (Sec. 5.2) as bench.py --editing times it: the terminal leaves of
    the ring's first camera (accumulated alpha beyond 0.99) over its whole 1920 x 1080 image,
    the paint of a seeded pattern (lowest ray wins), then the ring rendered in one launch with
    the edits active. The oracle finds every terminal leaf of that camera itself; the paint
    table must match its paint bit for bit, and sampled ring pixels its render with edits."""
    from oracle import editing as OE
    sc = scene_for_workload("forward")
    cams = ring_cameras(sc, 8, 1920, 1080, 40.0, 10.0, seed=2)
    t = float(np.random.default_rng(2002).uniform(0, sc.T))
    W, H = 1920, 1080
    n_cam = W * H
    n = 8 * n_cam
    tree = upload(sc)
    o = torch.empty(n, 3, device=DEV)
    d = torch.empty(n, 3, device=DEV)
    for i, cm in enumerate(cams):
        cs = _lib.make_camera(cm.width, cm.height, cm.fx, cm.fy, cm.cx, cm.cy, cm.c2w)
        _lib.neuvv_pinhole_rays(cs, n_cam, None, o[i * n_cam:(i + 1) * n_cam], d[i * n_cam:(i + 1) * n_cam])
    # the painting camera's rays as the oracle generates them, so both sides trace the same rays
    o0, d0 = OC.pinhole_rays(W, H, cams[0].intr(), cams[0].c2w)
    same = np.all(o[:n_cam].cpu().numpy() == o0, axis=1) & np.all(d[:n_cam].cpu().numpy() == d0, axis=1)
    assert same.mean() > 0.999, same.mean()
    o[:n_cam] = tdev(o0)
    d[:n_cam] = tdev(d0)
    announce(f"full size: terminal leaves of a {W}x{H} camera, {sc.n_leaves} leaves")
    last = torch.empty(n_cam, dtype=torch.int32, device=DEV)
    _lib.neuvv_find_terminal_leaves(tree.struct(), None, n_cam, o[:n_cam], d[:n_cam], None, t, W, 0.99, last)
    torch.cuda.synchronize()
    g = last.cpu().numpy().astype(np.int64)
    ref = oracle_render(sc, o0, d0, None, t, 0.01)          # stops where the alpha passes 0.99
    slots = tree.slot_of_input.cpu().numpy()
    amb = ref["margin"][:, 1] < 1e-4
    want = np.where(ref["last_leaf"] >= 0, slots[np.maximum(ref["last_leaf"], 0)], -1)
    announce(f"full-size terminal leaves: {int((want >= 0).sum())} rays pass 0.99, {int(amb.sum())} ambiguous")
    assert amb.sum() <= 0.002 * n_cam
    assert (want >= 0).sum() > 50_000
    assert np.array_equal(g[~amb], want[~amb])
    # paint with the stop-ambiguous rays left out on both sides
    colours = np.random.default_rng(2004).random((n_cam, 3)).astype(np.float32)
    g[amb] = -1
    tree.enable_edits()
    _lib.neuvv_paint(n_cam, torch.from_numpy(g.astype(np.int32)).to(DEV), tdev(colours), -1.0, 0.0, tree.n_leaves,
                     tree.edit)
    oe = OE.paint(OE.empty_edits(sc.n_leaves), np.where(amb, -1, ref["last_leaf"]), colours, -1.0, 0.0)
    torch.cuda.synchronize()
    ge = tree.edits_per_input().cpu().numpy().astype(np.float64)
    edited = np.isfinite(oe[:, 4])
    announce(f"full-size paint: {int(edited.sum())} leaves painted")
    assert edited.sum() > 10_000
    assert np.array_equal(np.isfinite(ge[:, 4]), edited)
    assert np.array_equal(ge[edited], oe[edited])
    assert np.all(ge[~edited, 3] == -1.0)
    # the ring with the edits active, in one launch
    rgb = torch.empty(n, 3, device=DEV)
    alpha = torch.empty(n, device=DEV)
    depth = torch.empty(n, device=DEV)
    nsamp = torch.empty(n, dtype=torch.int32, device=DEV)
    announce(f"full size: edited render of {n} rays")
    _lib.neuvv_render(tree.struct(), None, n, o, d, None, t, W, 1e-4, rgb, alpha, depth, nsamp)
    torch.cuda.synchronize()
    ns = nsamp.cpu().numpy()
    rng = np.random.default_rng(97)
    painted = np.nonzero(g >= 0)[0]
    hit = np.nonzero(ns > 0)[0]
    sample = np.unique(np.concatenate([rng.choice(painted, 800, replace=False), rng.choice(hit, 700, replace=False),
                                       rng.choice(n, 500, replace=False)]))
    cam_idx = sample // n_cam
    pix = (sample % n_cam).astype(np.int32)
    ro = np.zeros((sample.size, 3), np.float32)
    rd = np.zeros((sample.size, 3), np.float32)
    for cc in range(8):
        m = cam_idx == cc
        if m.any():
            ro[m], rd[m] = OC.pinhole_rays(W, H, cams[cc].intr(), cams[cc].c2w, pix[m])
    same = np.all(o[sample].cpu().numpy() == ro, axis=1) & np.all(d[sample].cpu().numpy() == rd, axis=1)
    assert same.mean() > 0.999, same.mean()
    sample, ro, rd = sample[same], ro[same], rd[same]
    vref = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, ro, rd, None, t, 1e-4, edit=oe)
    idx = torch.from_numpy(sample).to(DEV)
    gpu = dict(rgb=rgb[idx].cpu().numpy().astype(np.float64), alpha=alpha[idx].cpu().numpy().astype(np.float64),
               depth=depth[idx].cpu().numpy().astype(np.float64), nsamp=nsamp[idx].cpu().numpy())
    compare(gpu, vref, label="full-size edited ring")
    plain = oracle_render(sc, ro, rd, None, t, 1e-4)
    changed = (np.abs(vref["rgb"] - plain["rgb"]).max(1) > 1e-3).sum()
    announce(f"full-size edited ring: {int(changed)} of {sample.size} sampled pixels changed by the edits")
    assert changed > 500
