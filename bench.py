"""VOctree rendering benchmark on one MI355X.

Default workload: the forward-render configuration at full size: a depth-9
VOctree (~2M occupied leaves from 12 seeded ellipsoids forming a human-sized
blob), 16 HH coefficients x 3 channels + 8 density weights per leaf, density
basis [300 x 8], a ring of 8 cameras at 1920x1080 (16.6 M rays), one seeded
time per ring, FP32 storage, early stop at T < 1e-4. All inputs are seeded
and synthetic and resident in HBM before timing.

One step = the whole hot path over the ring: render forward (ray setup,
octree traversal, leaf evaluation, compositing, outputs) and the adjoint
(replay + atomic scatter into leaf coefficients and the density basis) for a
seeded upstream gradient. `value` = rays per step / step time (Mrays/s,
fwd+bwd); the forward-only rate is reported beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s fwd and fwd+bwd at 1080p; achieved HBM GB/s vs peak; PSNR vs FP64"
PEAK_HBM_GBS = 8000.0
FWD_RAY_IO_B = 24 + 24                      # o, d in; rgb, alpha, depth, nsamp out
BWD_RAY_NSAMP_B = 4                         # every ray: nsamp (rays without samples carry no gradient)
BWD_HIT_IO_B = 24 + 16 + 12                 # rays with samples: o, d; rgb, alpha; grad_rgb
TRACE_SAMPLE_B = {0: 32, 31: 48}            # traced step: trace bytes per sample (global form, per-point form)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(workload: str) -> str:
    """Hash of the sources the workload's render kernels are built from, comments and blank lines
    left out (a comment edit does not change the kernels)."""
    main = "render_pp.hip" if workload.endswith("per_point") else "render_kernels.h"
    h = hashlib.sha256()
    for f in (main, "render_common.h", "neuvv_device.h"):
        with open(os.path.join(ROOT, "paper_2202_06088_amd", "csrc", f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = [ln.split("//", 1)[0].rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None. kernel = "<name>/<layout>/<dtype>"."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(workload):
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", choices=["f32", "f16", "bf16"], default="f32")
    ap.add_argument("--layout", choices=["soa", "rows"], default="rows",
                    help="leaf payload layout: 16-byte-vector SoA or leaf-major rows")
    ap.add_argument("--form", choices=["global", "per-point"], default="global",
                    help="global: K=16 HH, C=8 density weights, one hyperangle per frame; per-point: the "
                         "paper's 104-value leaf, K=14, C=31, Cg=31 with the per-point hyperangle")
    ap.add_argument("--lighting", action="store_true",
                    help="also time the spotlight shadow + falloff pass (light map, low-pass, shading)")
    ap.add_argument("--editing", action="store_true",
                    help="also time appearance editing: terminal leaves + paint from one camera, and the forward "
                         "render with the edits active")
    ap.add_argument("--multi", type=int, default=0,
                    help="also time the exact merge of this many (2..4) interpenetrating placements of the tree")
    ap.add_argument("--no-trace", action="store_true",
                    help="time neuvv_render + neuvv_render_backward (the adjoint walks again) instead of the traced "
                         "pair (the adjoint replays the forward's per-sample trace)")
    ap.add_argument("--workload", choices=["ring", "train", "mixed", "multi"], default="ring",
                    help="ring: the forward-render ring (the default line). train: the differentiable training "
                         "step (depth 8, 65,536 random rays, per-ray t, L2 loss). mixed: depth-10 stereo 2048x2048 "
                         "per eye, forward at FP32 / FP16 / BF16 storage. multi: four depth-9 FP16 trees placed "
                         "and re-timed, rendered as layers, composed (Alg. 1) and differentiated")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.workload != "ring":
        return workload_bench(args)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}). "
              "Rays are independent, so N GPUs would each render a share of the ring; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_06088_amd import _lib, ops
    from paper_2202_06088_amd.voctree import VOctree
    from workloads import WORKLOADS, make_scene_per_point, ring_cameras, scene_for_workload

    dt = {"f32": _lib.F32, "f16": _lib.F16, "bf16": _lib.BF16}[args.dtype]
    t0 = time.time()
    log(f"generating the depth-9 humanoid scene (seeded, {args.form} hyperangle)")
    if args.form == "global":
        sc = scene_for_workload("forward")
    else:
        c2 = WORKLOADS["forward"]
        sc = make_scene_per_point(c2["depth"], c2["target"], c2["kind"], T=c2["T"], seed=c2["seed"])
    cams = ring_cameras(sc, 8, 1920, 1080, 40.0, 10.0, seed=2)
    t_frame = float(np.random.default_rng(2002).uniform(0, sc.T))
    log(f"scene: {sc.n_leaves} leaves, T={sc.T}, t={t_frame:.3f} ({time.time() - t0:.1f}s)")
    dev = "cuda"
    layout = _lib.LAYOUT_VEC_SOA if args.layout == "soa" else _lib.LAYOUT_LEAF_ROWS
    tree = VOctree.build(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, dt, dev, layout=layout,
                         wgam=sc.wgam, basis_g=sc.basis_g)
    W, H = 1920, 1080
    n_cam = W * H
    n = 8 * n_cam
    ray_o = torch.empty(n, 3, device=dev)
    ray_d = torch.empty(n, 3, device=dev)
    for i, c in enumerate(cams):
        cs = _lib.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.c2w)
        _lib.neuvv_pinhole_rays(cs, n_cam, None, ray_o[i * n_cam:(i + 1) * n_cam], ray_d[i * n_cam:(i + 1) * n_cam])
    rgb = torch.empty(n, 3, device=dev)
    alpha = torch.empty(n, device=dev)
    depth = torch.empty(n, device=dev)
    nsamp = torch.empty(n, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2003)
    g_rgb = torch.randn(n, 3, device=dev, generator=gen)
    grads = tree.zero_grads()
    stream = torch.cuda.current_stream()
    t_stop = 1e-4

    traced = not args.no_trace
    # trace room: one sample per ray covers the ring (0.69 per ray; a per-point sample takes two
    # 32-byte entries); a ray whose samples do not fit would be walked again by the adjoint
    trace_cap = n * (2 if tree.Cg > 0 else 1)
    trace = torch.empty(_lib.neuvv_trace_bytes(n, trace_cap), dtype=torch.uint8, device=dev) if traced else None

    def fwd():
        if traced:
            _lib.neuvv_render_trace(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth,
                                    nsamp, trace, trace_cap, stream)
        else:
            _lib.neuvv_render(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth,
                              nsamp, stream)

    def bwd():
        if traced:
            _lib.neuvv_render_backward_trace(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb,
                                             alpha, nsamp, g_rgb, None, grads[0], grads[1],
                                             grads[2] if tree.Cg > 0 else None, trace, trace_cap, stream)
        else:
            _lib.neuvv_render_backward(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha,
                                       nsamp, g_rgb, None, grads[0], grads[1], grads[2] if tree.Cg > 0 else None,
                                       stream)

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        fwd()
        bwd()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        fwd()
        ev[s][1].record(stream)
        bwd()
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - h0
    fwd_ms = float(np.mean([ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]))
    bwd_ms = float(np.mean([ev[s][1].elapsed_time(ev[s][2]) for s in range(args.steps)]))
    ms_step = wall * 1e3 / args.steps
    ns = nsamp.cpu().numpy().astype(np.int64)
    total_samples = int(ns.sum())
    hit = int((ns > 0).sum())
    values = 3 * tree.K + tree.C + tree.Cg                   # per sample: HH, density and hyperangle values
    payload_b = values * (4 if dt == _lib.F32 else 2)
    # leaves whose gradient row the adjoint changes (each row is read and written once)
    grads = tree.zero_grads()
    bwd()
    torch.cuda.synchronize()
    touched = int((grads[0][:, :values] != 0).any(dim=1).sum().item())
    elem = 4 if dt == _lib.F32 else 2
    # the adjoint: the leaf payload per sample (walking) or the trace entry (replaying); per touched
    # leaf its gradient row, read and written once, and its density and hyperangle weights (the
    # basis gradients are summed per leaf); per ray nsamp, per hit ray its inputs
    per_leaf = touched * (2 * 4 * values + (tree.C + tree.Cg) * elem)
    # the method's bytes (what Eq. 8 and its adjoint must move whatever the implementation): the
    # forward reads every sample's leaf payload once and every ray's input and output; the adjoint
    # needs every sample's payload again (its colour and density), each touched gradient row once
    # and the rays' inputs. The trace of the traced step is state this implementation keeps
    # between the passes (written by the forward, read by the adjoint in place of the payload):
    # reported beside, not counted.
    fwd_bytes = total_samples * payload_b + n * FWD_RAY_IO_B
    bwd_bytes = total_samples * payload_b + per_leaf + n * BWD_RAY_NSAMP_B + hit * BWD_HIT_IO_B
    trace_b = total_samples * TRACE_SAMPLE_B[tree.Cg] if traced else 0
    log(f"fwd {fwd_ms:.3f} ms, bwd {bwd_ms:.3f} ms per launch; step {ms_step:.3f} ms; "
        f"{total_samples} samples, {hit} hit rays")
    kern = {"render_fwd": (fwd_ms, fwd_bytes), "render_bwd": (bwd_ms, bwd_bytes)}
    dom = max(kern, key=lambda k: kern[k][0])
    workload = "forward_ring_d9_2M_8x1080p" + ("" if args.form == "global" else "_per_point")
    tkey = f"/{args.layout}/{args.dtype}{'/traced' if traced else ''}"

    def roof_of(k):
        ms, b = kern[k]
        traffic = measured_traffic(k + tkey, workload)
        r = {"kernel": k, "bound": "hbm", "achieved": round(b / (ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
             "unit": "GB/s", "frac": round(b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4), "traffic": traffic,
             "algorithmic_bytes_per_launch": b, "launch_ms": round(ms, 4),
             "trace_bytes_per_launch": trace_b}
        if traffic:
            # HBM bytes the counters saw (FETCH_SIZE + WRITE_SIZE, calibrated) over the same duration
            r["dram_gbs"] = round(traffic / (ms * 1e-3) / 1e9, 1)
            r["dram_frac"] = round(traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        return r

    roof = roof_of(dom)
    other = [k for k in kern if k != dom][0]
    roof_other = roof_of(other)
    # samples per ray over the rays that composited any (bins: 1, 2, 3-4, 5-8, ..., 129+)
    hs = ns[ns > 0]
    edges = [1, 2, 3, 5, 9, 17, 33, 65, 129, 1 << 30]
    hist = {f"{a}-{b - 1}" if b - 1 > a else f"{a}": int(((hs >= a) & (hs < b)).sum())
            for a, b in zip(edges[:-1], edges[1:])}
    hist = {k.replace(f"-{(1 << 30) - 1}", "+"): v for k, v in hist.items() if v}

    result = {
        "metric": METRIC, "value": round(n / (ms_step * 1e-3) / 1e6, 2), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": workload, "depth": sc.depth, "leaves": sc.n_leaves, "K": tree.K, "C": tree.C,
                   "Cg": tree.Cg,
                   "T": sc.T, "rays_per_step": n, "image": "8 x 1920x1080", "t_stop": t_stop,
                   "step": "render fwd + adjoint" + (" (traced)" if traced else ""), "layout": args.layout},
        "fwd_mrays_s": round(n / (fwd_ms * 1e-3) / 1e6, 2),
        "samples_per_step": total_samples, "hit_rays": hit, "leaves_touched": touched,
        "hit_fraction": round(hit / n, 5), "samples_per_hit_ray": round(total_samples / max(hit, 1), 3),
        "samples_per_ray_histogram": hist,
        "roofline": roof, "roofline_other_kernel": roof_other,
        "stream_ceiling": stream_ceiling(stream),
    }

    # the legs below compare against a plain forward (neuvv_render, no trace written)
    plain_fwd_ms = fwd_ms
    if traced and (args.lighting or args.multi or args.editing):
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record(stream)
        for _ in range(args.steps):
            _lib.neuvv_render(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth,
                              nsamp, stream)
        p1.record(stream)
        torch.cuda.synchronize()
        plain_fwd_ms = p0.elapsed_time(p1) / args.steps
        log(f"plain forward (no trace) {plain_fwd_ms:.3f} ms")
    if args.lighting:
        result["lighting"] = lighting_leg(sc, tree, ray_o, ray_d, rgb, alpha, depth, nsamp, t_frame, t_stop, W,
                                          plain_fwd_ms, stream, args.steps)
    if args.multi:
        if tree.Cg > 0 or not 2 <= args.multi <= 4:
            log("--multi needs the global form and 2..4 instances; skipped")
        else:
            result["multi"] = multi_leg(sc, tree, args.multi, ray_o, ray_d, t_frame, t_stop, W, plain_fwd_ms,
                                        stream, args.steps)
    if args.editing:
        if tree.Cg > 0:
            log("appearance edits are compiled for the global form only; --editing skipped")
        else:
            result["editing"] = editing_leg(tree, ray_o, ray_d, rgb, alpha, depth, nsamp, t_frame, t_stop, W, H,
                                            plain_fwd_ms, stream, args.steps)
    if not args.no_cpu_baseline:
        result.update(cpu_leg(sc, cams, t_frame, t_stop, rgb, g_rgb, grads, tree, args.cpu_seconds))
    print(json.dumps(result), flush=True)


def _timed(fn, steps, stream):
    """Average ms of fn() over steps calls, HIP events on the launch stream (after one warm call)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _sample_stats(nsamp_list):
    """Samples, hit rays and their ratios over the rays of one step (a list of nsamp tensors)."""
    s = sum(int(x.sum().item()) for x in nsamp_list)
    hit = sum(int((x > 0).sum().item()) for x in nsamp_list)
    n = sum(int(x.numel()) for x in nsamp_list)
    return {"samples_per_step": s, "hit_rays": hit, "hit_fraction": round(hit / max(n, 1), 5),
            "samples_per_hit_ray": round(s / max(hit, 1), 3)}


def _step_roofline(method_bytes, ms, parts):
    """The method's bytes of one step (the accounting of the main workload's roofline, summed over
    the step's calls) over the step time, against the HBM peak."""
    gbs = method_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "method_bytes_per_step": int(method_bytes), "achieved": round(gbs, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "parts": parts}


def _touched(grad_rows, values):
    """Leaves whose gradient row the adjoint changed."""
    return int((grad_rows[:, :values] != 0).any(dim=1).sum().item())


def workload_bench(args):
    """The other workloads (parity-tested in tests/test_gpu_workloads.py), timed with the library's calls:
    one JSON line each, value = rays per second of the timed unit."""
    import torch
    from paper_2202_06088_amd import _lib, ops
    from workloads import multi_instances, make_scene, orbit_camera, ring_cameras, scene_for_workload, stereo_cameras
    from paper_2202_06088_amd.voctree import VOctree
    if args.gpus != 1:
        log("one GPU only")
        sys.exit(2)
    dev = "cuda"
    stream = torch.cuda.current_stream()
    t_stop = 1e-4

    def upload(sc, dt):
        return VOctree.build(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, dt, dev)

    out = {"metric": METRIC, "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload == "train":
        sc = scene_for_workload("train")
        rng = np.random.default_rng(1003)
        tgt = type(sc)(sc.depth, sc.leaf_ijk, rng.normal(0, 0.3, sc.hh.shape).astype(np.float32), sc.wsig,
                       sc.basis, sc.gamma)
        cams = ring_cameras(sc, 8, 960, 540, 40.0, 10.0, seed=31) + ring_cameras(sc, 8, 960, 540, 40.0, -15.0,
                                                                                   seed=32)
        n = 65536
        ci = rng.integers(0, 16, n)
        pix = rng.integers(0, 960 * 540, n).astype(np.int32)
        o = torch.empty(n, 3, device=dev)
        d = torch.empty(n, 3, device=dev)
        for c in range(16):
            m = np.nonzero(ci == c)[0]
            cs = _lib.make_camera(960, 540, cams[c].fx, cams[c].fy, cams[c].cx, cams[c].cy, cams[c].c2w)
            oo, dd = ops.pinhole_rays(cs, torch.from_numpy(pix[m]).to(dev))
            idx = torch.from_numpy(m).to(dev)
            o[idx], d[idx] = oo, dd
        t = torch.from_numpy(rng.uniform(0, 300, n).astype(np.float32)).to(dev)
        tree, ttree = upload(sc, _lib.F32), upload(tgt, _lib.F32)
        target = ops.render(ttree, o, d, t, None, t_stop)[0]
        trace = ops.Trace(n, 16 * n, dev)           # room for every sample: the adjoint replays every ray
        grads = tree.zero_grads()

        def step():
            rgb, alpha, depth, nsamp = ops.render(tree, o, d, t, None, t_stop, trace=trace)
            g = 2.0 * (rgb - target)                     # d/dC of sum ||C - C*||^2 (Eq. 10)
            ops.render_backward(tree, o, d, rgb, alpha, nsamp, g, None, t, None, t_stop, grads=grads, trace=trace)

        for _ in range(args.warmup):
            step()
        ms = _timed(step, args.steps, stream)
        out.update(value=round(n / (ms * 1e-3) / 1e6, 2), ms_per_step=round(ms, 4), dtype="f32",
                   config={"workload": "train_d8_500k_65536rays", "leaves": sc.n_leaves, "rays_per_step": n,
                           "step": "traced render + L2 loss gradient + adjoint, per-ray t"})
        nsamp = ops.render(tree, o, d, t, None, t_stop)[3]
        st = _sample_stats([nsamp])
        values = 3 * tree.K + tree.C
        pay = values * 4
        touched = _touched(grads[0], values)
        # per-ray time: 4 more input bytes per ray in both calls
        fb = st["samples_per_step"] * pay + n * (FWD_RAY_IO_B + 4)
        bb = (st["samples_per_step"] * pay + touched * (2 * 4 * values + tree.C * 4) + n * BWD_RAY_NSAMP_B +
              st["hit_rays"] * (BWD_HIT_IO_B + 4))
        out.update(st)
        out["step_roofline"] = _step_roofline(fb + bb, ms, {"render": fb, "render_backward": bb,
                                                             "leaves_touched": touched})
        log(f"train: {ms:.3f} ms per step ({n} rays, {sc.n_leaves} leaves)")
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = train_cpu(sc, tgt, cams, ci, pix, t.cpu().numpy(), t_stop)
    elif args.workload == "mixed":
        sc = scene_for_workload("mixed")
        W = H = 2048
        eyes = stereo_cameras(sc, W, H, 90.0, seed=4)
        t = float(np.random.default_rng(4004).uniform(0, sc.T))
        # a stereo frame is one launch: the two eyes' rays stacked as one 2048 x 4096 image (the
        # tiles of 8 x 8 pixels never straddle the eyes), so that the hit rays of both share the GPU
        rays = [ops.pinhole_rays(_lib.make_camera(W, H, c.fx, c.fy, c.cx, c.cy, c.c2w)) for c in eyes]
        o2 = torch.cat([r[0] for r in rays])
        d2 = torch.cat([r[1] for r in rays])
        del rays
        n = 2 * W * H
        per = {}
        for name, dt in (("f32", _lib.F32), ("f16", _lib.F16), ("bf16", _lib.BF16)):
            tree = upload(sc, dt)
            buf = (torch.empty(n, 3, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev),
                   torch.empty(n, dtype=torch.int32, device=dev))

            def frame():
                ops.render(tree, o2, d2, t, None, t_stop, W, out=buf)

            for _ in range(args.warmup):
                frame()
            ms = _timed(frame, args.steps, stream)
            st = _sample_stats([buf[3]])
            mb = st["samples_per_step"] * (3 * tree.K + tree.C) * (4 if dt == _lib.F32 else 2) + n * FWD_RAY_IO_B
            per[name] = {"ms_per_stereo_frame": round(ms, 4), "mrays_s": round(n / (ms * 1e-3) / 1e6, 2),
                         "step_roofline": _step_roofline(mb, ms, {"render": mb})}
            if name == "f16":
                out.update(st)
            log(f"mixed {name}: {ms:.3f} ms per stereo frame")
            del tree
        out.update(value=per["f16"]["mrays_s"], ms_per_step=per["f16"]["ms_per_stereo_frame"], dtype="f16",
                   config={"workload": "mixed_d10_8M_stereo2048", "leaves": sc.n_leaves, "rays_per_step": n,
                           "step": "forward of one stereo frame (both eyes in one launch)", "per_dtype": per})
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = mixed_cpu(sc, eyes, W, H, t, t_stop)
    else:
        W, H = 1920, 1080
        scenes = [make_scene(9, 2_000_000, "human", K=16, C=8, T=300, seed=50 + i) for i in range(4)]
        G = scenes[0].G
        insts = [_lib.make_instance(p["rot"], p["trans"], p["scale"], p["time_offset"], p["wrap"])
                 for p in multi_instances(G, 4, seed=55)]
        cam = orbit_camera((0.0, 0.0, 0.45 * G), 3.2 * G, 0.4, 0.25, W, H, 50.0)
        o, d = ops.pinhole_rays(_lib.make_camera(W, H, cam.fx, cam.fy, cam.cx, cam.cy, cam.c2w))
        t = 37.5
        trees = [upload(s, _lib.F16) for s in scenes]
        grads = [tr.zero_grads() for tr in trees]
        gen = torch.Generator(device=dev)
        gen.manual_seed(5005)
        g_out = torch.randn(W * H, 3, device=dev, generator=gen)
        traces = [ops.Trace(W * H, 4 * W * H, dev) for _ in trees]   # room for every sample of a layer
        # the layers render into one stacked buffer, each on a stream of its own (default priority), so that
        # the four persistent launches overlap their tails; compose waits for all four, and the layers'
        # adjoints again run on their streams after it
        rgb_l = torch.empty(4, W * H, 3, device=dev)
        a_l = torch.empty(4, W * H, device=dev)
        d_l = torch.empty(4, W * H, device=dev)
        n_l = torch.empty(4, W * H, dtype=torch.int32, device=dev)
        sides = [torch.cuda.Stream() for _ in trees]

        def step():
            go = torch.cuda.Event()
            go.record(stream)
            done = []
            for i, (tr, ins, tc, sd) in enumerate(zip(trees, insts, traces, sides)):
                sd.wait_event(go)
                ops.render(tr, o, d, t, ins, t_stop, W, stream=sd, out=(rgb_l[i], a_l[i], d_l[i], n_l[i]), trace=tc)
                ev = torch.cuda.Event()
                ev.record(sd)
                done.append(ev)
            for ev in done:
                stream.wait_event(ev)
            ops.compose(rgb_l, a_l, d_l)
            g_rgb_l, g_a_l = ops.compose_backward(rgb_l, a_l, d_l, g_out, None)
            go2 = torch.cuda.Event()
            go2.record(stream)
            done = []
            for i, (tr, ins, sd) in enumerate(zip(trees, insts, sides)):
                sd.wait_event(go2)
                ops.render_backward(tr, o, d, rgb_l[i], a_l[i], n_l[i], g_rgb_l[i], g_a_l[i], t, ins, t_stop, W,
                                    grads=grads[i], trace=traces[i], stream=sd)
                ev = torch.cuda.Event()
                ev.record(sd)
                done.append(ev)
            for ev in done:
                stream.wait_event(ev)

        for _ in range(args.warmup):
            step()
        ms = _timed(step, args.steps, stream)
        n = W * H
        st = _sample_stats([n_l[i] for i in range(4)])
        values = 3 * trees[0].K + trees[0].C
        pay = values * 2
        touched = [_touched(g[0], values) for g in grads]
        hits = [int((n_l[i] > 0).sum().item()) for i in range(4)]
        fb = st["samples_per_step"] * pay + 4 * n * FWD_RAY_IO_B
        bb = (st["samples_per_step"] * pay + sum(touched) * (2 * 4 * values + trees[0].C * 2) +
              4 * n * BWD_RAY_NSAMP_B + sum(hits) * BWD_HIT_IO_B)
        # compose: rgb, alpha, depth of every layer in, one pixel out; its adjoint reads them and the
        # output gradient and writes the layers' rgb and alpha gradients
        cb = n * (4 * 20 + 20) + n * (4 * 20 + 12 + 4 * 16)
        out.update(st)
        out["step_roofline"] = _step_roofline(fb + bb + cb, ms, {"layer_renders": fb, "layer_adjoints": bb,
                                                                  "compose_and_adjoint": cb,
                                                                  "leaves_touched": touched})
        out.update(value=round(n / (ms * 1e-3) / 1e6, 2), ms_per_step=round(ms, 4), dtype="f16",
                   config={"workload": "multi_4xd9_1080p_fp16", "leaves": [s.n_leaves for s in scenes],
                           "rays_per_step": n,
                           "step": "4 traced layer renders + compose + compose adjoint + 4 replaying adjoints, "
                                   "the layers on 4 streams"})
        log(f"multi: {ms:.3f} ms per step (4 layers of {n} rays)")
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = multi_cpu(scenes, multi_instances(G, 4, seed=55), cam, W, H, t, t_stop)
    print(json.dumps(out), flush=True)


def _oracle_threads():
    from oracle import core as OC
    OC.build(force=False)
    return OC, OC.default_threads()


def train_cpu(sc, tgt, cams, ci, pix, t, t_stop):
    """The training step on the host: the FP64 oracle's forward of the step's rays, the L2 loss
    gradient against the oracle's target render, and the oracle's forward + gradient."""
    OC, threads = _oracle_threads()
    W, H = 960, 540
    o = np.zeros((pix.size, 3), np.float32)
    d = np.zeros((pix.size, 3), np.float32)
    for c in range(len(cams)):
        m = ci == c
        o[m], d[m] = OC.pinhole_rays(W, H, cams[c].intr(), cams[c].c2w, pix[m])
    target = OC.render(tgt.depth, tgt.leaf_ijk, tgt.hh, tgt.wsig, tgt.basis, tgt.gamma, o, d, t, 0.0, t_stop,
                       threads=threads)["rgb"]
    t0 = time.perf_counter()
    fwd = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, t, 0.0, t_stop, threads=threads)
    OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, t, 0.0, t_stop,
              g_rgb=2.0 * (fwd["rgb"] - target), threads=threads)
    dt = time.perf_counter() - t0
    log(f"train on the host: {pix.size} rays in {dt:.2f}s")
    return {"value": round(pix.size / dt / 1e6, 5), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"one step's {pix.size} rays: FP64 forward, loss gradient, forward + gradient",
            "host": OC.host_description()}


def mixed_cpu(sc, eyes, W, H, t, t_stop, stride=61):
    """The stereo frame's forward on the host: the FP64 oracle on every stride-th pixel of both eyes."""
    OC, threads = _oracle_threads()
    pix = np.arange(0, W * H, stride, dtype=np.int32)
    dt = 0.0
    for cam in eyes:
        o, d = OC.pinhole_rays(W, H, cam.intr(), cam.c2w, pix)
        t0 = time.perf_counter()
        OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, t, t_stop, threads=threads)
        dt += time.perf_counter() - t0
    n = 2 * pix.size
    log(f"mixed on the host: {n} rays in {dt:.2f}s")
    return {"value": round(n / dt / 1e6, 5), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th pixel of both eyes ({n} rays), FP64 forward on the unrounded payload",
            "host": OC.host_description()}


def multi_cpu(scenes, places, cam, W, H, t, t_stop, stride=31):
    """The multi-primitive step on the host for every stride-th pixel: the FP64 oracle's four
    layer renders, compose (Alg. 1) and its adjoint, and the four layers' forward + gradient."""
    OC, threads = _oracle_threads()
    pix = np.arange(0, W * H, stride, dtype=np.int32)
    o, d = OC.pinhole_rays(W, H, cam.intr(), cam.c2w, pix)
    insts = [OC.Instance(np.asarray(p["rot"], np.float32), np.asarray(p["trans"], np.float32), p["scale"],
                         p["time_offset"], p["wrap"]) for p in places]
    g_out = np.random.default_rng(5005).normal(size=(pix.size, 3))
    t0 = time.perf_counter()
    layers = [OC.render(s.depth, s.leaf_ijk, s.hh, s.wsig, s.basis, s.gamma, o, d, None, t, t_stop, inst,
                        threads=threads) for s, inst in zip(scenes, insts)]
    R = np.stack([l["rgb"] for l in layers]); A = np.stack([l["alpha"] for l in layers])
    D = np.stack([l["depth"] for l in layers])
    OC.compose(R, A, D)
    q_rgb, q_a = OC.compose_grad(R, A, D, g_out, np.zeros(pix.size))
    for i, (s, inst) in enumerate(zip(scenes, insts)):
        OC.render(s.depth, s.leaf_ijk, s.hh, s.wsig, s.basis, s.gamma, o, d, None, t, t_stop, inst,
                  g_rgb=q_rgb[i], g_alpha=q_a[i], threads=threads)
    dt = time.perf_counter() - t0
    log(f"multi on the host: {pix.size} pixels in {dt:.2f}s")
    return {"value": round(pix.size / dt / 1e6, 5), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th pixel ({pix.size} pixels): FP64 layer renders, compose and its adjoint, "
                      "layer forward + gradient, on the unrounded payload",
            "host": OC.host_description()}


def multi_leg(sc, tree, L, ray_o, ray_d, t_frame, t_stop, W, fwd_ms, stream, steps):
    """Exact merge of L interpenetrating placements of the tree on the ring: copies rotated about the
    vertical axis through the leaves' centroid by 2 pi k / (3 L) and shifted by a few percent of the
    grid, with time offsets 37 k; HIP events on the launch stream."""
    import torch
    from paper_2202_06088_amd import _lib
    c = sc.leaf_ijk.mean(0) + 0.5
    insts = []
    for k in range(L):
        th = 2 * math.pi * k / (3 * L)
        R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]], np.float32)
        trans = c - R @ c + np.array([0.04 * sc.G * k, -0.03 * sc.G * k, 0.0])
        insts.append(_lib.make_instance(R, trans, 1.0, 37.0 * k, 1))
    n = ray_o.shape[0]
    rgb = torch.empty(n, 3, device=ray_o.device)
    alpha = torch.empty(n, device=ray_o.device)
    depth = torch.empty(n, device=ray_o.device)
    nsamp = torch.empty(n, dtype=torch.int32, device=ray_o.device)
    trees = [tree.struct()] * L

    def once():
        _lib.neuvv_render_multi(trees, insts, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth, nsamp,
                                stream)

    once()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        once()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pieces = int(nsamp.sum())
    log(f"multi L={L}: {ms:.3f} ms ({n / ms / 1e3:.0f} Mrays/s), {pieces} pieces; single forward {fwd_ms:.3f} ms")
    return {"instances": L, "ms": round(ms, 4), "mrays_s": round(n / (ms * 1e-3) / 1e6, 2), "pieces": pieces,
            "vs_single_fwd": round(ms / fwd_ms, 3)}


def editing_leg(tree, ray_o, ray_d, rgb, alpha, depth, nsamp, t_frame, t_stop, W, H, fwd_ms, stream, steps):
    """Appearance editing (Sec. 5.2) on the ring: terminal leaves (alpha beyond 0.99) and paint
    of a seeded pattern from the first camera, then the ring's forward render with the edit
    table attached and active; HIP events on the launch stream."""
    import torch
    from paper_2202_06088_amd import _lib
    n_cam = W * H
    n = ray_o.shape[0]
    last = torch.empty(n_cam, dtype=torch.int32, device=ray_o.device)
    gen = torch.Generator(device=ray_o.device)
    gen.manual_seed(2004)
    colours = torch.rand(n_cam, 3, device=ray_o.device, generator=gen)
    tree.enable_edits()

    def paint_once():
        _lib.neuvv_find_terminal_leaves(tree.struct(), None, n_cam, ray_o[:n_cam], ray_d[:n_cam], None, t_frame, W,
                                        0.99, last, stream)
        _lib.neuvv_paint(n_cam, last, colours, -1.0, 0.0, tree.n_leaves, tree.edit, stream)

    def render_once():
        _lib.neuvv_render(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth, nsamp,
                          stream)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    paint_ms = timed(paint_once)
    painted = int((tree.edit[:, 4] == 0.0).sum())
    edited_ms = timed(render_once)
    tree.edit = None
    log(f"editing: paint one camera {paint_ms:.3f} ms ({painted} leaves); edited ring forward {edited_ms:.3f} ms "
        f"vs {fwd_ms:.3f} ms plain")
    return {"paint_one_camera_ms": round(paint_ms, 4), "painted_leaves": painted,
            "edited_forward_ms": round(edited_ms, 4), "overhead_vs_fwd": round(edited_ms / fwd_ms - 1.0, 4)}


def lighting_leg(sc, tree, ray_o, ray_d, rgb, alpha, depth, nsamp, t_frame, t_stop, W, fwd_ms, stream, steps):
    """Spotlight shadow and falloff (Sec. 5.2) over the ring: the light's alpha map (256 x 256,
    one forward launch), its Gaussian low-pass and the shading of every ring pixel; timed with
    HIP events on the launch stream, reported beside the forward render it adds to. Timed
    twice: the three calls one after the other, and a lit frame whose light map and low-pass
    run on a second stream (default priority) while the ring's forward render runs, the
    shading waiting for both; the frame's overhead is its time minus the plain forward's."""
    import torch
    from paper_2202_06088_amd import _lib, ops
    from workloads import look_at
    LW = LH = 256
    cen = sc.leaf_ijk.mean(0) + 0.5
    pos = cen + np.array([0.35 * sc.G, -0.25 * sc.G, 0.9 * sc.G])
    c2w = np.asarray(look_at(pos, cen), np.float32)
    f = 0.5 * LW / math.tan(math.radians(35.0))
    cam = _lib.make_camera(LW, LH, f, f, LW / 2, LH / 2, c2w)
    light = _lib.make_light(cam, float(sc.leaf_ijk[:, 2].min()), (0.7, 0.65, 0.6), (0.05, 0.1, 0.2), 0.8,
                            0.5 * sc.G)
    lo, ld = ops.pinhole_rays(cam)
    n = ray_o.shape[0]
    la = torch.empty(LW * LH, device=ray_o.device)
    lrgb = torch.empty(LW * LH, 3, device=ray_o.device)
    lns = torch.empty(LW * LH, dtype=torch.int32, device=ray_o.device)
    smap = torch.empty(LH, LW, device=ray_o.device)
    out = torch.empty(n, 3, device=ray_o.device)

    def once():
        _lib.neuvv_render(tree.struct(), None, LW * LH, lo, ld, None, t_frame, LW, t_stop, lrgb, la, None, lns,
                          stream)
        _lib.neuvv_blur(LH, LW, la, 1.5, smap, stream)
        _lib.neuvv_shade(light, smap, n, ray_o, ray_d, rgb, alpha, depth, out, stream)

    side = torch.cuda.Stream()
    go, lit_ready = torch.cuda.Event(), torch.cuda.Event()

    def lit_frame():
        go.record(stream)
        side.wait_event(go)
        _lib.neuvv_render(tree.struct(), None, LW * LH, lo, ld, None, t_frame, LW, t_stop, lrgb, la, None, lns,
                          side)
        _lib.neuvv_blur(LH, LW, la, 1.5, smap, side)
        lit_ready.record(side)
        _lib.neuvv_render(tree.struct(), None, n, ray_o, ray_d, None, t_frame, W, t_stop, rgb, alpha, depth,
                          nsamp, stream)
        stream.wait_event(lit_ready)
        _lib.neuvv_shade(light, smap, n, ray_o, ray_d, rgb, alpha, depth, out, stream)

    ms = _timed(once, steps, stream)
    frame_ms = _timed(lit_frame, steps, stream)
    lit = int((la > 0.5).sum())
    log(f"lighting pass {ms:.3f} ms ({100 * ms / fwd_ms:.1f} % of the forward render); light map {lit} opaque px")
    log(f"lit frame {frame_ms:.3f} ms with the light map on a second stream: "
        f"{100 * (frame_ms / fwd_ms - 1.0):.1f} % over the forward render")
    return {"light_map": f"{LW}x{LH}", "sigma_px": 1.5, "ms": round(ms, 4), "overhead_vs_fwd": round(ms / fwd_ms, 4),
            "lit_frame_ms": round(frame_ms, 4), "lit_frame_overhead_vs_fwd": round(frame_ms / fwd_ms - 1.0, 4),
            "light_map_opaque_px": lit}


def cpu_leg(sc, cams, t_frame, t_stop, rgb_gpu, g_rgb, grads, tree, budget_s):
    """FP64 oracle (as written, untuned) on a strided sample of the ring's rays, forward +
    gradient, on the host cores; also the GPU's error against it on those rays."""
    from oracle import core as OC
    W, H = 1920, 1080
    n_cam = W * H
    n_all = 8 * n_cam
    threads = OC.default_threads()
    OC.build(force=False)

    def run(stride, offset=0, threads=threads):
        g_idx = np.arange(offset, n_all, stride, dtype=np.int64)
        cam_of = g_idx // n_cam
        o = np.zeros((g_idx.size, 3), np.float32)
        d = np.zeros((g_idx.size, 3), np.float32)
        for c in range(8):
            m = cam_of == c
            if m.any():
                o[m], d[m] = OC.pinhole_rays(W, H, cams[c].intr(), cams[c].c2w, (g_idx[m] % n_cam).astype(np.int32))
        g = g_rgb[torch_index(g_idx, g_rgb.device)].cpu().numpy().astype(np.float64)
        t1 = time.perf_counter()
        ref = OC.render(sc.depth, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, t_frame, t_stop,
                        g_rgb=g, threads=threads, wgam=sc.wgam, basis_g=sc.basis_g)
        return g_idx, ref, time.perf_counter() - t1

    log(f"cpu baseline pilots ({threads} threads)")
    n_a, _, t_a = run(n_all // 64)          # fixed cost (hash set of the leaves, thread start)
    n_b, _, t_b = run(257)
    rate = max((len(n_b) - len(n_a)) / max(t_b - t_a, 1e-3), 1.0)
    stride = max(1, int(n_all / max(rate * budget_s, 1.0)))
    log(f"pilot rate {rate / 1e6:.3f} Mrays/s; sample stride {stride}")
    g_idx, ref, dt = run(stride, 1)
    gpu = rgb_gpu[torch_index(g_idx, rgb_gpu.device)].cpu().numpy().astype(np.float64)
    ok = ref["margin"][:, 1] >= 1e-4
    err = np.abs(gpu - ref["rgb"])[ok]
    mse = float(np.mean(err ** 2)) if err.size else 0.0
    psnr = 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")
    log(f"oracle {len(g_idx)} rays fwd+grad in {dt:.2f}s; GPU max-abs {err.max(initial=0):.3e} PSNR {psnr:.1f} dB")
    # one core: the same oracle on a smaller strided sample (~a third of the budget)
    stride1 = max(1, int(n_all / max(rate / threads * budget_s / 3, 1.0)))
    g1, _, dt1 = run(stride1, 2, threads=1)
    log(f"oracle on 1 thread: {len(g1)} rays in {dt1:.2f}s")
    return {
        "cpu_baseline": {"value": round(len(g_idx) / dt / 1e6, 5), "unit": "Mrays/s", "cores": threads,
                         "kind": "oracle",
                         "sample": (f"every {stride}th ray of" if stride > 1 else "all rays of") +
                                   f" the 8-camera ring ({len(g_idx)} rays), FP64 forward + gradient",
                         "one_core_value": round(len(g1) / dt1 / 1e6, 5),
                         "one_core_sample": f"every {stride1}th ray of the ring ({len(g1)} rays)",
                         "host": OC.host_description()},
        "psnr_vs_fp64_db": None if math.isinf(psnr) else round(psnr, 2),
        "maxabs_vs_fp64": float(f"{err.max(initial=0):.3e}"),
        "fp64_compare_rays": int(ok.sum()),
    }


def torch_index(idx, device):
    import torch
    return torch.from_numpy(idx).to(device)


def stream_ceiling(stream, nbytes=1 << 30, reps=10):
    """Measured streaming rates on this GPU beside the 8 TB/s datasheet peak: a 1 GiB
    device-to-device copy (read + write bytes) and a read-only pass (a sum over 1 GiB), HIP
    events on the launch stream."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    r = torch.empty((), device="cuda")
    out = {}
    for name, fn, moved in (("copy_gbs", lambda: b.copy_(a), 2 * nbytes),
                            ("read_gbs", lambda: torch.sum(a, 0, out=r), nbytes)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    log(f"stream ceiling: copy {out['copy_gbs']} GB/s, read {out['read_gbs']} GB/s")
    return out


def calibrate_copy(nbytes=1 << 30):
    """A plain device-to-device copy of known size, for scaling HBM byte counters."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {nbytes} bytes 3 times")


if __name__ == "__main__":
    main()
