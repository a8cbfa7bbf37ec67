"""Full-size parity of the training, mixed-precision and multi-primitive workloads.

* training step: depth-8 humanoid (~500k leaves), 65,536 rays drawn from 16
  seeded cameras at 960x540 with per-ray t in [0, 300), L2 loss against a
  target render of a second payload draw; forward + adjoint against FP64.
* mixed precision: depth-10 humanoid (~8M leaves), stereo 2048x2048 per eye,
  both eyes in one launch as the benchmark renders a stereo frame, FP16 / BF16 / FP32 leaf storage; per image (4 seeded frames x 2 eyes) the
  max-abs error and PSNR of rgb over the whole image against the FP64 oracle
  on the unrounded payload, and parity on the rounded payload, on a seeded
  pixel sample.
* multi-primitive: 4 depth-9 trees under seeded rotations, scales 0.5-2 and
  looping time offsets 0-150, FP16 storage, 1920x1080: render, compose,
  compose adjoint and the 4 render adjoints, against the oracle on sampled
  pixels (gradients restricted to those pixels).
"""
import math

import numpy as np
import pytest
import torch

from gpu_util import DEV, announce, compare, oracle_render, rel_err, round_storage, stop_ambiguous, tdev, upload
from oracle import core as OC
from paper_2202_06088_amd import _lib, ops
from workloads import (multi_instances, make_scene, orbit_camera, ring_cameras, scene_for_workload,
                       stereo_cameras)

pytestmark = pytest.mark.gpu


def test_training_step_full_size():
    sc = scene_for_workload("train")
    announce(f"training step: {sc.n_leaves} leaves")
    rng = np.random.default_rng(1003)
    tgt_hh = rng.normal(0, 0.3, sc.hh.shape).astype(np.float32)
    cams = ring_cameras(sc, 8, 960, 540, 40.0, 10.0, seed=31) + ring_cameras(sc, 8, 960, 540, 40.0, -15.0, seed=32)
    n = 65536
    ci = rng.integers(0, 16, n)
    pix = rng.integers(0, 960 * 540, n).astype(np.int32)
    t = rng.uniform(0, 300, n).astype(np.float32)
    o = torch.empty(n, 3, device=DEV)
    d = torch.empty(n, 3, device=DEV)
    ro = np.zeros((n, 3), np.float32)
    rd = np.zeros((n, 3), np.float32)
    for c in range(16):
        m = np.nonzero(ci == c)[0]
        cs = _lib.make_camera(960, 540, cams[c].fx, cams[c].fy, cams[c].cx, cams[c].cy, cams[c].c2w)
        oo, dd = ops.pinhole_rays(cs, tdev(pix[m], torch.int32))
        idx = torch.from_numpy(m).to(DEV)
        o[idx], d[idx] = oo, dd
        ro[m], rd[m] = OC.pinhole_rays(960, 540, cams[c].intr(), cams[c].c2w, pix[m])
    assert np.array_equal(o.cpu().numpy(), ro)
    same = np.all(d.cpu().numpy() == rd, axis=1)
    assert same.mean() > 0.999
    tree = upload(sc)
    target_scene = type(sc)(sc.depth, sc.leaf_ijk, tgt_hh, sc.wsig, sc.basis, sc.gamma)
    tgt_tree = upload(target_scene)
    tt = tdev(t)
    target, _, _, _ = ops.render(tgt_tree, o, d, tt, None, 1e-4)
    # oracle on the same rays, its own target and loss gradient
    ref_t = oracle_render(target_scene, ro, rd, t, 0.0, 1e-4)
    ref_f = oracle_render(sc, ro, rd, t, 0.0, 1e-4)
    amb = stop_ambiguous(ref_f, ref_t, label="train") | ~same
    gC = 2.0 * (ref_f["rgb"] - ref_t["rgb"])
    gC[amb] = 0.0
    ref = oracle_render(sc, ro, rd, t, 0.0, 1e-4, g_rgb=gC)
    amb_dev = torch.from_numpy(amb).to(DEV)
    # the plain calls, then the traced pair exactly as the benchmark's training step runs it
    # (trace room for sixteen samples per ray, the loss gradient from the traced forward's output)
    for traced in (False, True):
        trace = ops.Trace(n, 16 * n, DEV) if traced else None
        announce(f"training step, traced={traced}")
        rgb, alpha, depth, nsamp = ops.render(tree, o, d, tt, None, 1e-4, trace=trace)
        g = 2.0 * (rgb - target)                     # d/dC of sum ||C - C*||^2 (Eq. 10)
        g[amb_dev] = 0.0
        gl, gb = ops.render_backward(tree, o, d, rgb, alpha, nsamp, g.contiguous(), None, tt, None, 1e-4,
                                     trace=trace)
        torch.cuda.synchronize()
        gpu = dict(rgb=rgb.cpu().numpy().astype(np.float64), alpha=alpha.cpu().numpy().astype(np.float64),
                   depth=depth.cpu().numpy().astype(np.float64), nsamp=nsamp.cpu().numpy())
        if traced:   # the room holds every sample with margin: the adjoint replays every ray
            assert 2 * int(gpu["nsamp"].sum()) <= trace.cap, (int(gpu["nsamp"].sum()), trace.cap)
        compare({k: v[same] for k, v in gpu.items()}, {k: v[same] for k, v in ref_f.items()},
                label=f"train fwd traced={traced}")
        hh, ws = tree.unpack_grad(gl)
        e = [rel_err(hh.cpu().numpy(), ref["grad_hh"]), rel_err(ws.cpu().numpy(), ref["grad_wsig"]),
             rel_err(gb.cpu().numpy(), ref["grad_basis"])]
        announce(f"training step traced={traced} adjoint rel errors {e}")
        assert max(e) <= 1e-4


def test_mixed_precision_stereo_full_size():
    """Both eyes in one launch, stacked as one 2048 x 4096 image (the benchmark's stereo frame);
    errors are taken per eye image."""
    sc = scene_for_workload("mixed")
    announce(f"mixed precision: {sc.n_leaves} leaves, depth {sc.depth}")
    W = H = 2048
    eyes = stereo_cameras(sc, W, H, 90.0, seed=4)
    frames = np.random.default_rng(4004).uniform(0, sc.T, 4)
    rng = np.random.default_rng(4005)
    trees = {dt: upload(sc, dt) for dt in (_lib.F32, _lib.F16, _lib.BF16)}
    gpu_rays = [ops.pinhole_rays(_lib.make_camera(W, H, c.fx, c.fy, c.cx, c.cy, c.c2w)) for c in eyes]
    o = torch.cat([r[0] for r in gpu_rays])
    d = torch.cat([r[1] for r in gpu_rays])
    host_rays, same_eye = [], []
    for ei, cam in enumerate(eyes):
        ro, rd = OC.pinhole_rays(W, H, cam.intr(), cam.c2w)
        same = np.all(gpu_rays[ei][0].cpu().numpy() == ro, axis=1) & np.all(gpu_rays[ei][1].cpu().numpy() == rd, axis=1)
        assert same.mean() > 0.999
        host_rays.append((ro, rd))
        same_eye.append(same)
    report = []
    for t in frames:
        outs = {dt: ops.render(tr, o, d, float(t), None, 1e-4, W) for dt, tr in trees.items()}
        torch.cuda.synchronize()
        for ei, ((ro, rd), same) in enumerate(zip(host_rays, same_eye)):
            eye = slice(ei * W * H, (ei + 1) * W * H)
            # the whole image against FP64 on the unrounded payload: per image max-abs and PSNR of
            # rgb over every pixel except those whose stop decision is within rounding of t_stop
            # (counted) and the few whose GPU ray differs from the oracle's in the last bit
            announce(f"eye {ei} t={t:.2f}: FP64 oracle over all {W * H} pixels")
            ref64 = oracle_render(sc, ro, rd, None, float(t), 1e-4)
            ok = same & (ref64["margin"][:, 1] >= 1e-4)
            assert (~ok).sum() <= 0.002 * ok.size, int((~ok).sum())
            for dt, (rgb, alpha, depth, nsamp) in outs.items():
                err = np.abs(rgb[eye].cpu().numpy().astype(np.float64) - ref64["rgb"])[ok]
                mse = float(np.mean(err ** 2))
                psnr = 10 * math.log10(1.0 / mse) if mse > 0 else math.inf
                report.append((ei, float(t), dt, float(err.max()), psnr, int((~ok).sum())))
                if dt == _lib.F16:
                    assert err.max() <= 2e-3
                if dt == _lib.F32:
                    assert err.max() <= 1e-5 * max(np.abs(ref64["rgb"]).max(), 1e-30)
            del ref64
            # 16-bit storage on the rounded payload (the arithmetic alone), on a seeded pixel sample
            ns = outs[_lib.F32][3][eye].cpu().numpy()
            hit = np.nonzero((ns > 0) & same)[0]
            pix = np.unique(np.concatenate([rng.choice(hit, min(1500, hit.size), replace=False),
                                            rng.choice(np.nonzero(same)[0], 300, replace=False)])).astype(np.int64)
            pidx = torch.from_numpy(pix + ei * W * H).to(DEV)
            for dt in (_lib.F16, _lib.BF16):
                rgb, alpha, depth, nsamp = outs[dt]
                g = dict(rgb=rgb[pidx].cpu().numpy().astype(np.float64),
                         alpha=alpha[pidx].cpu().numpy().astype(np.float64),
                         depth=depth[pidx].cpu().numpy().astype(np.float64), nsamp=nsamp[pidx].cpu().numpy())
                compare(g, oracle_render(sc, ro[pix], rd[pix], None, float(t), 1e-4, dtype=dt),
                        label=f"eye{ei} t={t:.1f} dtype{dt} vs rounded")
    for r in report:
        announce(f"eye {r[0]} t={r[1]:.2f} storage {['f32', 'f16', 'bf16'][r[2]]}: whole image max-abs "
                 f"{r[3]:.3e} PSNR {r[4]:.1f} dB ({r[5]} pixels excluded)")


def test_multi_primitive_composition_full_size():
    W, H = 1920, 1080
    scenes = [make_scene(9, 2_000_000, "human", K=16, C=8, T=300, seed=50 + i) for i in range(4)]
    G = scenes[0].G
    places = multi_instances(G, 4, seed=55)
    insts = [(OC.Instance(p["rot"], p["trans"], p["scale"], p["time_offset"], p["wrap"]),
              _lib.make_instance(p["rot"], p["trans"], p["scale"], p["time_offset"], p["wrap"])) for p in places]
    cam = orbit_camera((0.0, 0.0, 0.45 * G), 3.2 * G, 0.4, 0.25, W, H, 50.0)
    cs = _lib.make_camera(W, H, cam.fx, cam.fy, cam.cx, cam.cy, cam.c2w)
    o, d = ops.pinhole_rays(cs)
    t = 37.5
    announce("multi-primitive: rendering 4 layers (traced, each on its own stream, as the benchmark's step)")
    trees = [upload(s, _lib.F16) for s in scenes]
    traces = [ops.Trace(W * H, 4 * W * H, DEV) for _ in trees]
    rgb_l = torch.empty(4, W * H, 3, device=DEV)
    a_l = torch.empty(4, W * H, device=DEV)
    d_l = torch.empty(4, W * H, device=DEV)
    n_l = torch.empty(4, W * H, dtype=torch.int32, device=DEV)
    main = torch.cuda.current_stream()
    sides = [torch.cuda.Stream() for _ in trees]
    go = torch.cuda.Event()
    go.record(main)
    for i, (tr, ins, tc, sd) in enumerate(zip(trees, insts, traces, sides)):
        sd.wait_event(go)
        ops.render(tr, o, d, t, ins[1], 1e-4, W, stream=sd, out=(rgb_l[i], a_l[i], d_l[i], n_l[i]), trace=tc)
        ev = torch.cuda.Event()
        ev.record(sd)
        main.wait_event(ev)
    layers = [(rgb_l[i], a_l[i], d_l[i], n_l[i]) for i in range(4)]
    c_rgb, c_a, c_d = ops.compose(rgb_l, a_l, d_l)
    torch.cuda.synchronize()
    for l, tc in zip(layers, traces):   # the room holds every sample: the adjoints replay every ray
        assert 2 * int(l[3].sum()) <= tc.cap
    covered = np.nonzero(c_a.cpu().numpy() > 1e-3)[0]
    assert covered.size > 50_000
    rng = np.random.default_rng(56)
    pix = np.unique(np.concatenate([rng.choice(covered, 1200, replace=False),
                                    rng.choice(W * H, 200, replace=False)])).astype(np.int64)
    ro, rd = OC.pinhole_rays(W, H, cam.intr(), cam.c2w, pix.astype(np.int32))
    pidx = torch.from_numpy(pix).to(DEV)
    same = np.all(o[pidx].cpu().numpy() == ro, axis=1) & np.all(d[pidx].cpu().numpy() == rd, axis=1)
    assert same.mean() > 0.999
    pix, ro, rd = pix[same], ro[same], rd[same]
    pidx = torch.from_numpy(pix).to(DEV)
    refs = [oracle_render(s, ro, rd, None, t, 1e-4, inst=ins[0], dtype=_lib.F16) for s, ins in zip(scenes, insts)]
    amb = stop_ambiguous(*refs, label="multi-primitive layers")
    for i, r in enumerate(refs):
        g = dict(rgb=layers[i][0][pidx].cpu().numpy().astype(np.float64),
                 alpha=layers[i][1][pidx].cpu().numpy().astype(np.float64),
                 depth=layers[i][2][pidx].cpu().numpy().astype(np.float64),
                 nsamp=layers[i][3][pidx].cpu().numpy())
        compare(g, r, label=f"layer {i}")
    R = np.stack([r["rgb"] for r in refs]); A = np.stack([r["alpha"] for r in refs])
    Dp = np.stack([r["depth"] for r in refs])
    # depth order decided on GPU depths for near-equal layer depths is not unique: skip those pixels
    order_amb = np.zeros(pix.size, bool)
    for i in range(4):
        for j in range(i + 1, 4):
            fin = np.isfinite(Dp[i]) & np.isfinite(Dp[j])
            close = np.zeros(pix.size, bool)
            close[fin] = np.abs(Dp[i][fin] - Dp[j][fin]) <= 1e-4 * np.maximum(np.abs(Dp[i][fin]), 1.0)
            order_amb |= close
    keep = ~amb & ~order_amb
    announce(f"composite: {int(amb.sum())} stop-ambiguous and {int(order_amb.sum())} depth-tie pixels "
             f"of {pix.size} left out")
    r_rgb, r_a, r_d = OC.compose(R, A, Dp)
    # the composite, like each layer, to the FP32 forward bar
    e_rgb = rel_err(c_rgb[pidx].cpu().numpy()[keep], r_rgb[keep])
    e_a = rel_err(c_a[pidx].cpu().numpy()[keep], r_a[keep])
    announce(f"composite rel errors rgb {e_rgb:.2e} alpha {e_a:.2e}")
    assert e_rgb <= 1e-5 and e_a <= 1e-5
    # adjoint: loss on the sampled composite pixels only
    gP = np.zeros((W * H, 3), np.float32)
    gA = np.zeros(W * H, np.float32)
    gvals = np.random.default_rng(57).normal(size=(pix.size, 3)).astype(np.float32)
    gavals = np.random.default_rng(58).normal(size=pix.size).astype(np.float32)
    gvals[~keep] = 0.0
    gavals[~keep] = 0.0
    gP[pix] = gvals
    gA[pix] = gavals
    announce("multi-primitive: compose and render adjoints")
    g_rgb_l, g_a_l = ops.compose_backward(rgb_l, a_l, d_l, tdev(gP), tdev(gA))
    q_rgb, q_a = OC.compose_grad(R, A, Dp, gvals.astype(np.float64), gavals.astype(np.float64))
    assert rel_err(g_rgb_l[:, pidx].cpu().numpy(), q_rgb) <= 1e-4
    assert rel_err(g_a_l[:, pidx].cpu().numpy(), q_a) <= 1e-4
    grads = [tr.zero_grads() for tr in trees]   # zeroed on the main stream before the side streams wait
    go2 = torch.cuda.Event()
    go2.record(main)
    for i, (tr, ins, sd) in enumerate(zip(trees, insts, sides)):
        sd.wait_event(go2)
        l = layers[i]
        ops.render_backward(tr, o, d, l[0], l[1], l[3], g_rgb_l[i], g_a_l[i], t, ins[1], 1e-4, W,
                            grads=grads[i], trace=traces[i], stream=sd)
    torch.cuda.synchronize()
    for i, (tr, ins, s) in enumerate(zip(trees, insts, scenes)):
        gl, gb = grads[i][0], grads[i][1]
        ref = oracle_render(s, ro, rd, None, t, 1e-4, inst=ins[0], dtype=_lib.F16, g_rgb=q_rgb[i], g_alpha=q_a[i])
        hh, ws = tr.unpack_grad(gl)
        e = [rel_err(hh.cpu().numpy(), ref["grad_hh"]), rel_err(ws.cpu().numpy(), ref["grad_wsig"]),
             rel_err(gb.cpu().numpy(), ref["grad_basis"])]
        announce(f"tree {i} adjoint rel errors {e}")
        assert max(e) <= 1e-4
