"""Differentiable rendering: a torch.autograd.Function over render_views / render_views_backward.

Gradients of an image loss flow to the transfer-function control-point RGBA values (positions
fixed) and, for lod-0 views of an octree whose level-0 nodes all hold bricks, to the level-0
voxel values.  Torch only provides memory, streams and the autograd graph; the forward (which
records the transmittance before every position it evaluates) and the adjoint are the HIP
kernels behind the C ABI.
"""
from __future__ import annotations

import copy

import torch

from .octree import Octree


class RenderFn(torch.autograd.Function):
    """images = RenderFn.apply(tf_rgba, voxels, tree, views)

    tf_rgba: [n_views][C][8][4] float32 tensor -- overrides each view's control-point RGBA
    voxels:  None, or a tensor standing for the level-0 volume the tree was built from
             ([C][Dz][Dy][Dx] float32); its gradient is produced when it requires grad
    Returns one [H][W][4] float32 CUDA image per view."""

    @staticmethod
    def forward(ctx, tf_rgba, voxels, tree: Octree, views):
        vs = []
        rgba = tf_rgba.detach().to("cpu", torch.float32).numpy()
        for i, v in enumerate(views):
            w = copy.copy(v)
            w.tf_rgba = rgba[i].copy()
            vs.append(w)
        ckpt = torch.empty(max(tree.ckpt_bytes(vs), 1), dtype=torch.uint8, device="cuda")
        imgs = tree.render(vs, ckpt=ckpt)
        ctx.tree, ctx.views, ctx.ckpt = tree, vs, ckpt
        ctx.want_vox = voxels is not None and voxels.requires_grad
        ctx.tf_device = tf_rgba.device
        ctx.vox_shape = tuple(voxels.shape) if voxels is not None else None
        return tuple(imgs)

    @staticmethod
    def backward(ctx, *grads):
        tree, vs = ctx.tree, ctx.views
        g = [gr.contiguous().float() if gr is not None else
             torch.zeros((v.height, v.width, 4), dtype=torch.float32, device="cuda")
             for gr, v in zip(grads, vs)]
        dctrl = torch.zeros((len(vs), tree.C, 8, 4), dtype=torch.float32, device="cuda")
        dvox = None
        if ctx.want_vox:
            Dx, Dy, Dz = tree.dims
            dvox = torch.zeros((tree.C, Dz, Dy, Dx), dtype=torch.float32, device="cuda")
        tree.render_backward(vs, g, ctx.ckpt, dctrl, dvox)
        return dctrl.to(ctx.tf_device), dvox, None, None


def render(tree: Octree, views, tf_rgba: torch.Tensor, voxels: torch.Tensor | None = None):
    """Differentiable render; see RenderFn."""
    return RenderFn.apply(tf_rgba, voxels, tree, views)
