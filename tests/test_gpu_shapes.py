"""GPU parity of every compiled leaf shape of the global-hyperangle form:
K in {14, 16, 30} HH functions per channel (Table 3's N = 14 and 30: all HH
functions with n <= 2 and n <= 3; the workloads' 16) times C in {8, 31}
density weights (the workloads' 8, the paper's 31). For each: the forward on
a 64x64 view with early stop, and the adjoint (plain calls and traced pair)
against the FP64 oracle; K = 30 also with FP16 storage and per-ray time. The
full-size K = 30 ring is in test_gpu_fullsize.py."""
import math

import numpy as np
import pytest
import torch

from gpu_util import (announce, compare, gpu_render, oracle_render, rel_err, stop_ambiguous, tdev, tiny_camera,
                      upload)
from oracle import core as OC
from paper_2202_06088_amd import _lib, ops
from workloads import make_scene

pytestmark = pytest.mark.gpu

SHAPES = [(14, 8), (16, 8), (30, 8), (14, 31), (16, 31), (30, 31)]


def shape_scene(K, C):
    sc = make_scene(6, 20_000, "random", K=K, C=C, T=30, seed=40 + K + C)
    # density weights scaled by sqrt(8 / C): the logit keeps the spread it has with C = 8
    sc.wsig = (sc.wsig * math.sqrt(8.0 / C)).astype(np.float32)
    return sc


def _adjoint(tree, o, d, t, t_stop, gC, gA, traced):
    oo, dd = tdev(o), tdev(d)
    n = oo.shape[0]
    trace = ops.Trace(n, 2 * n, oo.device) if traced else None
    rgb, alpha, depth, nsamp = ops.render(tree, oo, dd, t, None, t_stop, 64, trace=trace)
    gl, gb = ops.render_backward(tree, oo, dd, rgb, alpha, nsamp, tdev(gC), tdev(gA), t, None, t_stop, 64,
                                 trace=trace)
    torch.cuda.synchronize()
    hh, ws = tree.unpack_grad(gl)
    pad = gl[:, 3 * tree.K + tree.C:]
    assert pad.numel() == 0 or float(pad.abs().max()) == 0.0, "row padding must stay zero"
    return hh.cpu().numpy(), ws.cpu().numpy(), gb.cpu().numpy()


@pytest.mark.parametrize("K,C", SHAPES)
def test_shape_forward_and_adjoint(K, C):
    sc = shape_scene(K, C)
    tree = upload(sc)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    announce(f"shape K={K} C={C}: forward")
    ref = oracle_render(sc, o, d, None, 7.25, 1e-4)
    compare(gpu_render(tree, o, d, None, 7.25, 1e-4, image_width=64), ref, label=f"K={K} C={C}")
    rng = np.random.default_rng(K * 100 + C)
    gC = rng.normal(size=(o.shape[0], 3)).astype(np.float32)
    gA = rng.normal(size=o.shape[0]).astype(np.float32)
    amb = stop_ambiguous(ref, label=f"K={K} C={C}")
    gC[amb], gA[amb] = 0.0, 0.0
    gref = oracle_render(sc, o, d, None, 7.25, 1e-4, g_rgb=gC, g_alpha=gA)
    assert int(ref["nsamp"].sum()) > 3000
    for traced in (False, True):
        announce(f"shape K={K} C={C}: adjoint traced={traced}")
        gh, gw, gb = _adjoint(tree, o, d, 7.25, 1e-4, gC, gA, traced)
        e = [rel_err(gh, gref["grad_hh"]), rel_err(gw, gref["grad_wsig"]), rel_err(gb, gref["grad_basis"])]
        announce(f"K={K} C={C} traced={traced} grad rel errors {e}")
        assert max(e) <= 1e-4


def test_k30_fp16_and_per_ray_time():
    sc = shape_scene(30, 8)
    tree16 = upload(sc, _lib.F16)
    tree = upload(sc)
    rng = np.random.default_rng(3008)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    announce("K=30: FP16 storage against the rounded payload and the unrounded one")
    compare(gpu_render(tree16, o, d, None, 4.0, 1e-4, image_width=64),
            oracle_render(sc, o, d, None, 4.0, 1e-4, dtype=_lib.F16), label="K=30 f16 vs rounded")
    g = gpu_render(tree16, o, d, None, 4.0, 1e-4, image_width=64)
    r64 = oracle_render(sc, o, d, None, 4.0, 1e-4)
    ok = r64["margin"][:, 1] >= 1e-4
    err = np.abs(g["rgb"] - r64["rgb"])[ok].max()
    announce(f"K=30 FP16 max-abs vs unrounded {err:.2e}")
    assert err <= 2e-3
    t = rng.uniform(0, 29, o.shape[0]).astype(np.float32)
    gC = rng.normal(size=(o.shape[0], 3)).astype(np.float32)
    gA = rng.normal(size=o.shape[0]).astype(np.float32)
    fwd = oracle_render(sc, o, d, t, 0.0, 1e-4)
    compare(gpu_render(tree, o, d, t, 0.0, 1e-4, image_width=64), fwd, label="K=30 per-ray t")
    amb = stop_ambiguous(fwd, label="K=30 per-ray t")
    gC[amb], gA[amb] = 0.0, 0.0
    gref = oracle_render(sc, o, d, t, 0.0, 1e-4, g_rgb=gC, g_alpha=gA)
    for traced in (False, True):
        gh, gw, gb = _adjoint(tree, o, d, tdev(t), 1e-4, gC, gA, traced)
        e = [rel_err(gh, gref["grad_hh"]), rel_err(gw, gref["grad_wsig"]), rel_err(gb, gref["grad_basis"])]
        announce(f"K=30 per-ray t traced={traced} grad rel errors {e}")
        assert max(e) <= 1e-4
