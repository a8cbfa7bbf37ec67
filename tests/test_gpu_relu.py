"""GPU parity of the ReLU density activation (Eq. 5 as the paper prints it; the
softplus of the other tests is the workloads' reading): forward and adjoint of
the K = 16, C = 8 form (plain and traced pair, FP32 and FP16 storage, early
stop on and off) and of the paper's per-point leaf (K = 14, C = 31, Cg = 31),
against the FP64 oracle with the same activation. With ReLU a leaf whose
density logit is negative is transparent, so the scenes have both kinds."""
import numpy as np
import pytest
import torch

from gpu_util import (announce, compare, gpu_render, oracle_render, rel_err, stop_ambiguous, tdev, tiny_camera,
                      upload)
from oracle import core as OC
from paper_2202_06088_amd import _lib, ops
from workloads import make_scene_per_point, random_rays, scene_for_workload

pytestmark = pytest.mark.gpu


def _grads(tree, o, d, t, t_stop, gC, gA, traced, image_width=64):
    oo, dd = tdev(o), tdev(d)
    n = oo.shape[0]
    room = (4 if tree.Cg > 0 else 2) * n
    trace = ops.Trace(n, room, oo.device) if traced else None
    rgb, alpha, depth, nsamp = ops.render(tree, oo, dd, t, None, t_stop, image_width, trace=trace)
    out = ops.render_backward(tree, oo, dd, rgb, alpha, nsamp, tdev(gC), tdev(gA), t, None, t_stop, image_width,
                              trace=trace)
    torch.cuda.synchronize()
    parts = tree.unpack_grad(out[0])
    return [p.cpu().numpy() for p in parts] + [g.cpu().numpy() for g in out[1:]]


@pytest.mark.parametrize("dtype", [_lib.F32, _lib.F16])
def test_relu_forward(dtype):
    sc = scene_for_workload("tiny")
    tree = upload(sc, dtype, density="relu")
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    for t, t_stop in ((4.0, 0.0), (7.25, 1e-4)):
        announce(f"relu forward dtype={dtype} t={t} t_stop={t_stop}")
        ref = oracle_render(sc, o, d, None, t, t_stop, dtype=dtype, density="relu")
        soft = oracle_render(sc, o, d, None, t, t_stop, dtype=dtype)
        assert np.abs(ref["alpha"] - soft["alpha"]).max() > 1e-2      # the activation matters here
        compare(gpu_render(tree, o, d, None, t, t_stop, image_width=64), ref, label=f"relu dtype={dtype} t={t}")


@pytest.mark.parametrize("traced", [False, True])
def test_relu_backward(traced):
    sc = scene_for_workload("tiny")
    tree = upload(sc, density="relu")
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    rng = np.random.default_rng(61)
    gC = rng.normal(size=(o.shape[0], 3)).astype(np.float32)
    gA = rng.normal(size=o.shape[0]).astype(np.float32)
    for t, t_stop in ((4.0, 0.0), (7.25, 1e-4)):
        fwd = oracle_render(sc, o, d, None, t, t_stop, density="relu")
        amb = stop_ambiguous(fwd, label=f"relu t={t}") if t_stop > 0 else np.zeros(o.shape[0], bool)
        g1, g2 = gC.copy(), gA.copy()
        g1[amb], g2[amb] = 0.0, 0.0
        ref = oracle_render(sc, o, d, None, t, t_stop, g_rgb=g1, g_alpha=g2, density="relu")
        announce(f"relu backward traced={traced} t={t} t_stop={t_stop}")
        gh, gw, gb = _grads(tree, o, d, t, t_stop, g1, g2, traced)
        e = [rel_err(gh, ref["grad_hh"]), rel_err(gw, ref["grad_wsig"]), rel_err(gb, ref["grad_basis"])]
        announce(f"relu traced={traced} t={t} grad rel errors {e}")
        assert max(e) <= 1e-4
        # leaves the oracle gives no gradient (negative logit: transparent) get none on the GPU either
        dead = np.all(ref["grad_hh"].reshape(ref["grad_hh"].shape[0], -1) == 0, axis=1)
        assert np.all(gh.reshape(gh.shape[0], -1)[dead] == 0.0)


def test_relu_per_point_leaf():
    """The paper's 104-value leaf with Eq. 5's ReLU: forward, and the traced adjoint with one
    time for every ray and with a time per ray."""
    sc = make_scene_per_point(6, 20_000, "random", T=30, seed=31)
    tree = upload(sc, density="relu")
    rng = np.random.default_rng(62)
    cam = tiny_camera(sc)
    o, d = OC.pinhole_rays(64, 64, cam.intr(), cam.c2w)
    announce("relu per-point forward")
    compare(gpu_render(tree, o, d, None, 7.25, 1e-4, image_width=64),
            oracle_render(sc, o, d, None, 7.25, 1e-4, density="relu"), label="relu per-point")
    gC = rng.normal(size=(o.shape[0], 3)).astype(np.float32)
    gA = rng.normal(size=o.shape[0]).astype(np.float32)
    names = ["grad_hh", "grad_wsig", "grad_wgam", "grad_basis", "grad_basis_g"]
    for per_ray in (False, True):
        t = rng.uniform(0, 29, o.shape[0]).astype(np.float32) if per_ray else 12.5
        fwd = oracle_render(sc, o, d, t if per_ray else None, 0.0 if per_ray else t, 1e-4, density="relu")
        amb = stop_ambiguous(fwd, label=f"relu per-point per_ray={per_ray}")
        g1, g2 = gC.copy(), gA.copy()
        g1[amb], g2[amb] = 0.0, 0.0
        ref = oracle_render(sc, o, d, t if per_ray else None, 0.0 if per_ray else t, 1e-4, g_rgb=g1, g_alpha=g2,
                            density="relu")
        announce(f"relu per-point traced backward per_ray={per_ray}")
        gpu = _grads(tree, o, d, tdev(t) if per_ray else t, 1e-4, g1, g2, True)
        e = [rel_err(g, ref[n]) for g, n in zip(gpu, names)]
        announce(f"relu per-point per_ray={per_ray} grad rel errors {e}")
        assert max(e) <= 1e-4
