"""torch.autograd.Function over the HIP forward render and its hand-written backward.

    img = render(means, scales, quats, opacities, sh, cams, rasterizer)   # [V,H,W,3]
    loss = (img - target).abs().mean(); loss.backward()

`scales` and `opacities` are the activated values (apply exp / sigmoid in torch
before calling, and autograd carries the chain). The forward keeps the per-view
records and tile lists for the backward (the rasterizer hands those buffers
over and allocates new ones for later calls), so several renders may be alive
at once.
"""
from __future__ import annotations

import torch

from .raster import DeviceScene, Rasterizer, ViewBatch


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, cams, rz: Rasterizer):
        ds = DeviceScene(*(t.detach().contiguous() for t in (means, scales, quats, opacities, sh)))
        vb = rz.render_views(ds, cams)
        # the records, lists and per-pixel state stay with this node for the
        # backward; the rasterizer's later calls get new buffers
        rz.release()
        keep = ViewBatch(V=vb.V, N=vb.N, proj=vb.proj, tiles_touched=vb.tiles_touched,
                         order=None, n_pairs=vb.n_pairs, sorted_ids=vb.sorted_ids[: max(vb.n_pairs, 1)],
                         tile_ranges=vb.tile_ranges, image=None, p_final=vb.p_final,
                         t_final=vb.t_final, n_walk=vb.n_walk)
        ctx.rz, ctx.cams, ctx.vb, ctx.ds = rz, cams, keep, ds
        return vb.image

    @staticmethod
    def backward(ctx, grad_image):
        grads = ctx.rz.backward(ctx.ds, ctx.vb, ctx.cams, grad_image.contiguous())
        return grads["means"], grads["scales"], grads["quats"], grads["opacities"], grads["sh"], None, None


def render(means, scales, quats, opacities, sh, cams, rz: Rasterizer) -> torch.Tensor:
    """Differentiable render of views that share one image size: [V, H, W, 3]."""
    return RenderFunction.apply(means, scales, quats, opacities, sh, cams, rz)
