"""Shared helpers of the GPU parity tests: upload a seeded scene to the
library, round payloads the way 16-bit storage does (on the oracle side, in
numpy), and compare a GPU render against the FP64 oracle."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

from oracle import core as OC
from paper_2202_06088_amd import _lib, ops
from paper_2202_06088_amd.voctree import VOctree

DEV = "cuda"


def announce(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def tdev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def upload(scene, dtype=_lib.F32, layout=_lib.LAYOUT_LEAF_ROWS, density="softplus") -> VOctree:
    return VOctree.build(scene.depth, scene.leaf_ijk, scene.hh, scene.wsig, scene.basis, scene.gamma, dtype,
                         layout=layout, wgam=scene.wgam, basis_g=scene.basis_g,
                         density=_lib.DENSITY_RELU if density == "relu" else _lib.DENSITY_SOFTPLUS)


def round_storage(x: np.ndarray, dtype: int) -> np.ndarray:
    """Round-to-nearest-even of float32 values to the storage type, returned as float64."""
    x = np.ascontiguousarray(x, np.float32)
    if dtype == _lib.F32:
        return x.astype(np.float64)
    if dtype == _lib.F16:
        with np.errstate(over="ignore"):   # beyond the largest float16: +-inf, as the format rounds
            return x.astype(np.float16).astype(np.float64)
    # bfloat16 keeps the top 16 bits of the float32 pattern: add half an ulp of
    # the kept part minus one, plus the kept part's lowest bit (ties to even),
    # then truncate. A carry out of the mantissa moves the exponent, which is
    # the correct rounding (up to +inf past the largest finite value). NaN stays
    # NaN (the addition could carry a NaN pattern into the sign bit).
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    with np.errstate(invalid="ignore"):
        out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[np.isnan(x)] = np.nan
    return out


def oracle_render(scene, o, d, t=None, t_scalar=0.0, t_stop=1e-4, inst=None, dtype=_lib.F32, g_rgb=None,
                  g_alpha=None, density="softplus"):
    wg = None if scene.wgam is None else round_storage(scene.wgam, dtype)
    return OC.render(scene.depth, scene.leaf_ijk, round_storage(scene.hh, dtype), round_storage(scene.wsig, dtype),
                     scene.basis, scene.gamma, o, d, t, t_scalar, t_stop, inst, g_rgb, g_alpha, wgam=wg,
                     basis_g=scene.basis_g, density=density)


def gpu_render(tree, o, d, t=None, t_scalar=0.0, t_stop=1e-4, inst=None, image_width=0):
    tt = tdev(t) if t is not None else t_scalar
    rgb, alpha, depth, nsamp = ops.render(tree, tdev(o), tdev(d), tt, inst, t_stop, image_width)
    torch.cuda.synchronize()
    return dict(rgb=rgb.cpu().numpy().astype(np.float64), alpha=alpha.cpu().numpy().astype(np.float64),
                depth=depth.cpu().numpy().astype(np.float64), nsamp=nsamp.cpu().numpy())


def inst_pair(rot, trans, scale, off, wrap):
    """(oracle Instance, C-ABI neuvv_instance) for the same float32 placement."""
    return (OC.Instance(np.asarray(rot, np.float32), np.asarray(trans, np.float32), scale, off, wrap),
            _lib.make_instance(rot, trans, scale, off, wrap))


def compare(gpu, ref, tol=1e-5, delta_margin=1e-5, stop_margin=1e-4, max_ambiguous=0.002, label=""):
    """FP32 GPU render against the FP64 oracle.

    rgb and alpha: max |gpu - ref| <= tol * max |ref| over all rays except those
    whose early-stop test fell within stop_margin (relative) of t_stop, where
    the two precisions may legitimately stop at different samples.
    nsamp: identical except on those rays and on rays whose smallest sampled
    segment is shorter than delta_margin leaf units (a crossing within rounding
    of a cell edge). depth: relative tol where alpha > 1e-4; +inf exactly where
    nothing was sampled. Returns the statistics."""
    m = ref["margin"]
    stop_amb = m[:, 1] < stop_margin
    delta_amb = m[:, 0] < delta_margin
    ok = ~stop_amb
    scale = max(np.abs(ref["rgb"]).max(), 1e-30)
    err_rgb = np.abs(gpu["rgb"] - ref["rgb"])[ok].max(initial=0.0)
    err_a = np.abs(gpu["alpha"] - ref["alpha"])[ok].max(initial=0.0)
    a_scale = max(np.abs(ref["alpha"]).max(), 1e-30)
    sure = ok & ~delta_amb
    ns_bad = int((gpu["nsamp"][sure] != ref["nsamp"][sure]).sum())
    hitd = ok & (ref["alpha"] > 1e-4)
    fin = ref["depth"][hitd]
    dscale = max(np.abs(fin).max(initial=0.0), 1e-30)
    err_d = np.abs(gpu["depth"][hitd] - fin).max(initial=0.0)
    empty = ref["nsamp"] == 0
    stats = dict(n=len(ok), stop_ambiguous=int(stop_amb.sum()), delta_ambiguous=int(delta_amb.sum()),
                 rel_rgb=err_rgb / scale, rel_alpha=err_a / a_scale, rel_depth=err_d / dscale, nsamp_mismatch=ns_bad,
                 hit=int((ref["nsamp"] > 0).sum()))
    announce(f"{label} {stats}")
    assert stats["rel_rgb"] <= tol, stats
    assert stats["rel_alpha"] <= tol, stats
    assert stats["rel_depth"] <= tol, stats
    assert ns_bad == 0, stats
    assert np.all(np.isinf(gpu["depth"][empty & sure])), "empty rays must have infinite depth"
    assert (stop_amb.sum() + delta_amb.sum()) <= max(2, max_ambiguous * len(ok)), stats
    return stats


def stop_ambiguous(*refs, margin=1e-4, max_frac=0.002, label=""):
    """Rays whose early-stop test, in any of the oracle renders refs, fell within margin
    (relative) of t_stop: FP32 and FP64 may stop at different samples there, so gradient tests
    give those rays no upstream gradient. The same 1e-4 as the forward's bar; the count is
    printed and held to max_frac of the rays (at least 2)."""
    amb = np.zeros(refs[0]["margin"].shape[0], bool)
    for r in refs:
        amb |= r["margin"][:, 1] < margin
    n_amb = int(amb.sum())
    announce(f"{label} stop-ambiguous rays excluded from the gradient: {n_amb} of {amb.size}")
    assert n_amb <= max(2, max_frac * amb.size), (n_amb, amb.size)
    return amb


def rel_err(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).max(initial=0.0) /
                 max(np.abs(np.asarray(b, np.float64)).max(initial=0.0), 1e-30))


def tiny_camera(scene, seed=11):
    from workloads import orbit_camera
    """64x64 pinhole, hfov 30 degrees, seeded direction, 2.5 G from the centroid of the leaves."""
    rng = np.random.default_rng(seed)
    G = scene.G
    ctr = scene.leaf_ijk.mean(0) + 0.5
    return orbit_camera(ctr, 2.5 * G, rng.uniform(0, 2 * math.pi), rng.uniform(-0.5, 0.5), 64, 64, 30.0)


def cam_struct(cam):
    return _lib.make_camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.c2w)
