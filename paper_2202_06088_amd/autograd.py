"""torch.autograd wrappers: the forward saves only rgb, alpha and nsamp per
ray; the backward kernel replays the compositing with the transmittance
recomputed (Sec. 4.3 "Optimization")."""
from __future__ import annotations

import torch

from . import _lib, ops
from .voctree import VOctree


class RenderFn(torch.autograd.Function):
    """rgb, alpha, depth, nsamp = RenderFn.apply(hh, wsig, basis, tree, ray_o, ray_d, t, inst, t_stop, image_width)

    hh, wsig, basis must be the float32 tensors the tree renders from
    (tree.hh, tree.wsig, tree.basis): their gradients come back in the same
    packed layout, ready for an element-wise optimizer step."""

    @staticmethod
    def forward(ctx, hh, wsig, basis, tree: VOctree, ray_o, ray_d, t, inst, t_stop, image_width):
        if tree.dtype != _lib.F32:
            raise ValueError("autograd needs float32 leaf storage; call ops.render_backward for 16-bit trees")
        if hh.data_ptr() != tree.hh.data_ptr() or wsig.data_ptr() != tree.wsig.data_ptr() \
                or basis.data_ptr() != tree.basis.data_ptr():
            raise ValueError("hh / wsig / basis must be the tree's own tensors")
        rgb, alpha, depth, nsamp = ops.render(tree, ray_o, ray_d, t, inst, t_stop, image_width)
        ctx.tree, ctx.inst, ctx.t_stop, ctx.image_width = tree, inst, t_stop, image_width
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
        gl, gb = ops.render_backward(ctx.tree, ray_o, ray_d, rgb, alpha, nsamp, g_rgb.contiguous(),
                                     None if g_alpha is None else g_alpha.contiguous(), t_arg, ctx.inst,
                                     ctx.t_stop, ctx.image_width, want_basis=ctx.needs_input_grad[2])
        ghh, gws = ctx.tree.rows_to_payload_f32(gl)
        return ghh, gws, (gb if ctx.needs_input_grad[2] else None), None, None, None, None, None, None, None


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
    return RenderFn.apply(tree.hh, tree.wsig, tree.basis, tree, ray_o, ray_d, t, inst, t_stop, image_width)


def compose(rgb, alpha, depth):
    return ComposeFn.apply(rgb, alpha, depth)
