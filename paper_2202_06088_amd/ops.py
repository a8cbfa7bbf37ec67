"""Functional front end over the C ABI: allocates the output tensors and
calls the library. Every computation runs in the HIP kernels."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _lib
from .voctree import VOctree


def _dev(x: torch.Tensor):
    if not x.is_cuda:
        raise ValueError("device tensors required")
    return x.device


def _arg(name: str, x, dtype=torch.float32, shape=None, optional: bool = False):
    """The library reads raw pointers: each tensor argument must be a contiguous device tensor
    of the expected dtype and shape (None entries of `shape` are free)."""
    if x is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if x.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None:
        if x.dim() != len(shape) or any(w is not None and w != g for w, g in zip(shape, x.shape)):
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")


def _rays(ray_o, ray_d, t):
    n = ray_o.shape[0] if isinstance(ray_o, torch.Tensor) else -1
    _arg("ray_o", ray_o, shape=(n, 3))
    _arg("ray_d", ray_d, shape=(n, 3))
    if isinstance(t, torch.Tensor):
        _arg("t", t, shape=(n,))
    return n


class Trace:
    """Per-sample trace of one forward call (neuvv_render_trace), replayed by the adjoint of the
    same call (neuvv_render_backward_trace). Room for `cap` 32-byte entries (a sample takes one in
    the K = 16, C = 8 form and two in the per-point form); rays whose samples do not fit are
    walked again by the adjoint."""

    def __init__(self, n_rays: int, cap: int, device):
        self.n_rays = int(n_rays)
        self.cap = int(cap)
        self.buf = torch.empty(_lib.neuvv_trace_bytes(self.n_rays, self.cap), dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0


def render(tree: VOctree, ray_o: torch.Tensor, ray_d: torch.Tensor, t=0.0, inst: Optional[_lib.neuvv_instance] = None,
           t_stop: float = 1e-4, image_width: int = 0, want_depth: bool = True, stream=None, out=None,
           trace: Optional[Trace] = None):
    """Returns (rgb [n,3], alpha [n], depth [n] or None, nsamp [n] int32); with a Trace the call
    also records its samples there."""
    n = _rays(ray_o, ray_d, t)
    dev = _dev(ray_o)
    ray_t = t if isinstance(t, torch.Tensor) else None
    t_scalar = 0.0 if ray_t is not None else float(t)
    if out is None:
        rgb = torch.empty(n, 3, device=dev)
        alpha = torch.empty(n, device=dev)
        depth = torch.empty(n, device=dev) if want_depth else None
        nsamp = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        rgb, alpha, depth, nsamp = out
        _arg("rgb", rgb, shape=(n, 3))
        _arg("alpha", alpha, shape=(n,))
        _arg("depth", depth, shape=(n,), optional=True)
        _arg("nsamp", nsamp, torch.int32, shape=(n,))
    if trace is not None:
        if trace.n_rays != n:
            raise ValueError(f"the trace was made for {trace.n_rays} rays, not {n}")
        _lib.neuvv_render_trace(tree.struct(), inst, n, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb,
                                alpha, depth, nsamp, trace.buf, trace.cap, stream)
    else:
        _lib.neuvv_render(tree.struct(), inst, n, ray_o, ray_d, ray_t, t_scalar, image_width, t_stop, rgb, alpha,
                          depth, nsamp, stream)
    return rgb, alpha, depth, nsamp


def render_backward(tree: VOctree, ray_o, ray_d, rgb, alpha, nsamp, grad_rgb, grad_alpha=None, t=0.0,
                    inst=None, t_stop: float = 1e-4, image_width: int = 0, grads=None, want_basis=True,
                    stream=None, trace: Optional[Trace] = None):
    """Accumulates into float32 buffers (fresh zeros if grads is None) and returns them:
    (grad_leaf [N, ROW], grad_basis [T, C]), plus grad_basis_g [T, Cg] for a tree with
    per-point hyperangle weights. With the Trace of the forward call, replays its samples."""
    n = _rays(ray_o, ray_d, t)
    _arg("rgb", rgb, shape=(n, 3))
    _arg("alpha", alpha, shape=(n,))
    _arg("nsamp", nsamp, torch.int32, shape=(n,))
    _arg("grad_rgb", grad_rgb, shape=(n, 3))
    _arg("grad_alpha", grad_alpha, shape=(n,), optional=True)
    if grads is None:
        grads = tree.zero_grads()
    gl, gb = grads[0], grads[1]
    gbg = grads[2] if tree.Cg > 0 else None
    _arg("grad_leaf", gl, shape=(tree.n_leaves, tree.grad_row))
    _arg("grad_basis", gb, shape=(tree.T, tree.C))
    _arg("grad_basis_g", gbg, shape=(tree.T, tree.Cg), optional=True)
    ray_t = t if isinstance(t, torch.Tensor) else None
    t_scalar = 0.0 if ray_t is not None else float(t)
    if trace is not None:
        if trace.n_rays != n:
            raise ValueError(f"the trace was made for {trace.n_rays} rays, not {n}")
        _lib.neuvv_render_backward_trace(tree.struct(), inst, ray_o.shape[0], ray_o, ray_d, ray_t, t_scalar,
                                         image_width, t_stop, rgb, alpha, nsamp, grad_rgb, grad_alpha, gl,
                                         gb if want_basis else None, gbg if want_basis else None, trace.buf,
                                         trace.cap, stream)
    else:
        _lib.neuvv_render_backward(tree.struct(), inst, ray_o.shape[0], ray_o, ray_d, ray_t, t_scalar, image_width,
                                   t_stop, rgb, alpha, nsamp, grad_rgb, grad_alpha, gl, gb if want_basis else None,
                                   gbg if want_basis else None, stream)
    return (gl, gb, gbg) if tree.Cg > 0 else (gl, gb)


def compose(rgb: torch.Tensor, alpha: torch.Tensor, depth: torch.Tensor, stream=None):
    """rgb [L,n,3], alpha [L,n], depth [L,n] -> (rgb [n,3], alpha [n], depth [n])."""
    L, n = alpha.shape
    _arg("rgb", rgb, shape=(L, n, 3))
    _arg("alpha", alpha, shape=(L, n))
    _arg("depth", depth, shape=(L, n))
    dev = _dev(rgb)
    o_rgb = torch.empty(n, 3, device=dev)
    o_a = torch.empty(n, device=dev)
    o_d = torch.empty(n, device=dev)
    _lib.neuvv_compose(L, n, rgb, alpha, depth, o_rgb, o_a, o_d, stream)
    return o_rgb, o_a, o_d


def compose_backward(rgb, alpha, depth, grad_out_rgb, grad_out_alpha=None, stream=None):
    L, n = alpha.shape
    _arg("rgb", rgb, shape=(L, n, 3))
    _arg("alpha", alpha, shape=(L, n))
    _arg("depth", depth, shape=(L, n))
    _arg("grad_out_rgb", grad_out_rgb, shape=(n, 3))
    _arg("grad_out_alpha", grad_out_alpha, shape=(n,), optional=True)
    g_rgb = torch.empty_like(rgb)
    g_a = torch.empty_like(alpha)
    _lib.neuvv_compose_backward(L, n, rgb, alpha, depth, grad_out_rgb, grad_out_alpha, g_rgb, g_a, stream)
    return g_rgb, g_a


def pinhole_rays(cam: _lib.neuvv_camera, pix: Optional[torch.Tensor] = None, device="cuda", stream=None):
    n = cam.width * cam.height if pix is None else pix.shape[0]
    _arg("pix", pix, torch.int32, shape=(n,), optional=True)
    o = torch.empty(n, 3, device=device)
    d = torch.empty(n, 3, device=device)
    _lib.neuvv_pinhole_rays(cam, n, pix, o, d, stream)
    return o, d


def eval_hh(K: int, dirs: torch.Tensor, gam: torch.Tensor, stream=None):
    _arg("dirs", dirs, shape=(None, 3))
    _arg("gam", gam, shape=(dirs.shape[0],))
    out = torch.empty(dirs.shape[0], K, device=dirs.device)
    _lib.neuvv_eval_hh(K, dirs.shape[0], dirs, gam, out, stream)
    return out


def blur(img: torch.Tensor, sigma: float, stream=None):
    """Gaussian low-pass of a [H, W] float32 map (the shadow map, Sec. 5.2)."""
    H, W = img.shape
    img = img.contiguous()
    _arg("img", img, shape=(H, W))
    out = torch.empty_like(img)
    _lib.neuvv_blur(H, W, img, sigma, out, stream)
    return out


def shade(light: _lib.neuvv_light, shadow_map: Optional[torch.Tensor], ray_o, ray_d, rgb, alpha, depth, stream=None):
    """Viewer colour [n, 3] of a rendered layer over the lit ground (shadow and falloff, Sec. 5.2)."""
    n = _rays(ray_o, ray_d, None)
    _arg("shadow_map", shadow_map, shape=(light.camera.height, light.camera.width), optional=True)
    _arg("rgb", rgb, shape=(n, 3))
    _arg("alpha", alpha, shape=(n,))
    _arg("depth", depth, shape=(n,))
    out = torch.empty_like(rgb)
    _lib.neuvv_shade(light, shadow_map, ray_o.shape[0], ray_o, ray_d, rgb, alpha, depth, out, stream)
    return out


def terminal_leaves(tree: VOctree, ray_o, ray_d, t=0.0, inst=None, alpha_threshold: float = 0.99,
                    image_width: int = 0, stream=None):
    """Leaf slot where each ray's accumulated alpha first exceeds the threshold, or -1 (Sec. 5.2)."""
    n = _rays(ray_o, ray_d, t)
    out = torch.empty(n, dtype=torch.int32, device=_dev(ray_o))
    ray_t = t if isinstance(t, torch.Tensor) else None
    t_scalar = 0.0 if ray_t is not None else float(t)
    _lib.neuvv_find_terminal_leaves(tree.struct(), inst, n, ray_o, ray_d, ray_t, t_scalar, image_width,
                                    alpha_threshold, out, stream)
    return out


def paint(tree: VOctree, last_leaf: torch.Tensor, colours: torch.Tensor, sigma_d: float = -1.0, t_d: float = 0.0,
          stream=None):
    """Writes the target colours into the tree's edit table at the rays' terminal leaves."""
    colours = colours.contiguous()
    _arg("last_leaf", last_leaf, torch.int32, shape=(None,))
    _arg("colours", colours, shape=(last_leaf.shape[0], 3))
    if tree.edit is None:
        tree.enable_edits()
    _lib.neuvv_paint(last_leaf.shape[0], last_leaf, colours, sigma_d, t_d, tree.n_leaves, tree.edit,
                     stream)
    return tree.edit
