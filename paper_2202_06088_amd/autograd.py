"""torch.autograd wrappers: the forward saves rgb, alpha and nsamp per ray
and a trace of its samples with room for two per ray; the backward kernel
replays the compositing with the transmittance
recomputed (Sec. 4.3 "Optimization"), from the trace where it holds the ray."""
from __future__ import annotations

import torch

from . import _lib, ops
from .voctree import VOctree


class RenderFn(torch.autograd.Function):
    """rgb, alpha, depth, nsamp = RenderFn.apply(hh, wsig, basis, wgam, basis_g, tree, ray_o, ray_d, t, inst,
    t_stop, image_width)

    hh, wsig, basis (and wgam, basis_g for a tree with per-point hyperangle weights, else
    None) must be the float32 tensors the tree renders from: their gradients come back in the
    same packed layout, ready for an element-wise optimizer step."""

    @staticmethod
    def forward(ctx, hh, wsig, basis, wgam, basis_g, tree: VOctree, ray_o, ray_d, t, inst, t_stop, image_width):
        if tree.dtype != _lib.F32:
            raise ValueError("autograd needs float32 leaf storage; call ops.render_backward for 16-bit trees")
        own = [(hh, tree.hh), (wsig, tree.wsig), (basis, tree.basis)]
        if tree.Cg > 0:
            own += [(wgam, tree.wgam), (basis_g, tree.basis_g)]
        if any(a is None or a.data_ptr() != b.data_ptr() for a, b in own):
            raise ValueError("the payload and basis tensors must be the tree's own")
        n = ray_o.shape[0]
        # room for two samples per ray (a per-point sample takes two entries)
        trace = ops.Trace(n, (4 if tree.Cg > 0 else 2) * n, ray_o.device) if 0 < n < 2 ** 29 else None
        rgb, alpha, depth, nsamp = ops.render(tree, ray_o, ray_d, t, inst, t_stop, image_width, trace=trace)
        ctx.tree, ctx.inst, ctx.t_stop, ctx.image_width, ctx.trace = tree, inst, t_stop, image_width, trace
        ctx.t_scalar = None if isinstance(t, torch.Tensor) else float(t)
        ctx.save_for_backward(ray_o, ray_d, rgb, alpha, nsamp, t if isinstance(t, torch.Tensor) else None)
        ctx.mark_non_differentiable(depth, nsamp)
        return rgb, alpha, depth, nsamp

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth, g_nsamp):
        ray_o, ray_d, rgb, alpha, nsamp, t = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        t_arg = t if t is not None else ctx.t_scalar
        tree = ctx.tree
        want_basis = ctx.needs_input_grad[2] or (tree.Cg > 0 and ctx.needs_input_grad[4])
        out = ops.render_backward(tree, ray_o, ray_d, rgb, alpha, nsamp, g_rgb.contiguous(),
                                  None if g_alpha is None else g_alpha.contiguous(), t_arg, ctx.inst,
                                  ctx.t_stop, ctx.image_width, want_basis=want_basis, trace=ctx.trace)
        ctx.trace = None
        parts = tree.rows_to_payload_f32(out[0])
        g_basis = out[1] if ctx.needs_input_grad[2] else None
        if tree.Cg > 0:
            g_wgam = parts[2]
            g_basis_g = out[2] if ctx.needs_input_grad[4] else None
        else:
            g_wgam = g_basis_g = None
        return (parts[0], parts[1], g_basis, g_wgam, g_basis_g) + (None,) * 7


class ComposeFn(torch.autograd.Function):
    """out_rgb, out_alpha, out_depth = ComposeFn.apply(rgb [L,n,3], alpha [L,n], depth [L,n])."""

    @staticmethod
    def forward(ctx, rgb, alpha, depth):
        rgb, alpha, depth = rgb.contiguous(), alpha.contiguous(), depth.contiguous()
        o_rgb, o_a, o_d = ops.compose(rgb, alpha, depth)
        ctx.save_for_backward(rgb, alpha, depth)
        ctx.mark_non_differentiable(o_d)
        return o_rgb, o_a, o_d

    @staticmethod
    def backward(ctx, g_rgb, g_a, g_d):
        rgb, alpha, depth = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros(rgb.shape[1:], device=rgb.device)
        gr, ga = ops.compose_backward(rgb, alpha, depth, g_rgb.contiguous(),
                                      None if g_a is None else g_a.contiguous())
        return gr, ga, None


def render(tree: VOctree, ray_o, ray_d, t=0.0, inst=None, t_stop=1e-4, image_width=0):
    return RenderFn.apply(tree.hh, tree.wsig, tree.basis, tree.wgam, tree.basis_g, tree, ray_o, ray_d, t, inst,
                          t_stop, image_width)


def compose(rgb, alpha, depth):
    return ComposeFn.apply(rgb, alpha, depth)
