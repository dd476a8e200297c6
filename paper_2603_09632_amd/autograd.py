"""Differentiation form: the rasterizer as a torch.autograd.Function.

forward  = xgs_project -> xgs_tile_sort -> xgs_render_fwd
backward = xgs_render_bwd, which recomputes each pixel's transmittance back to
           front from final_T instead of storing per-(pixel, Gaussian) state.

Saved for backward: the parameters, the projected splat records, the sorted
instance lists and ranges, final_T and n_last.  Opacity enters activated, so a
caller that optimises logits writes ``opacity=torch.sigmoid(raw)`` and torch
carries the chain rule through the sigmoid.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import (BWD_ALL, BWD_FEATURES_ONLY, Binning, Gaussians, Projected, XgsError, alloc_binning,
               camera_from, xgs_project, xgs_render_bwd, xgs_render_fwd, xgs_tile_sort)


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, colors, features, cam, max_instances, features_only):
        g = Gaussians(means.contiguous(), log_scales.contiguous(), quats.contiguous(), opacity.contiguous(),
                      colors.contiguous(), features.contiguous())
        c = camera_from(cam)
        p = xgs_project(g, c)
        if max_instances is None:
            max_instances = int(p.tiles_touched.to(torch.int64).sum().item())
        b = alloc_binning(g.n, max(int(max_instances), 1), c, means.device)
        xgs_tile_sort(p, c, g.n, b)
        out, final_T, n_last = xgs_render_fwd(g, p, b, c)
        ctx.cam = c
        ctx.features_only = bool(features_only)
        ctx.max_instances = b.max_instances
        ctx.save_for_backward(g.means, g.log_scales, g.quats, g.opacity, g.colors, g.features, p.splat,
                              p.radius, p.tile_rect, p.tiles_touched, b.keys, b.vals, b.ranges,
                              b.num_instances, b.status, b.tile_order, final_T, n_last)
        ctx.mark_non_differentiable(final_T, n_last)
        return out, final_T, n_last

    @staticmethod
    def backward(ctx, d_out, _d_final_T, _d_n_last):
        (means, log_scales, quats, opacity, colors, features, splat, radius, tile_rect, touched, keys, vals,
         ranges, num_inst, status, tile_order, final_T, n_last) = ctx.saved_tensors
        if int(status.item()) != 0:
            raise XgsError("render: the instance buffers overflowed in the forward pass")
        g = Gaussians(means, log_scales, quats, opacity, colors, features)
        p = Projected(splat, radius, tile_rect, touched)
        b = Binning(keys, vals, ranges, num_inst, status, torch.empty(1, dtype=torch.uint8, device=means.device),
                    ctx.max_instances, tile_order)
        flags = BWD_FEATURES_ONLY if ctx.features_only else BWD_ALL
        gr = xgs_render_bwd(g, p, b, ctx.cam, d_out.contiguous(), final_T, n_last, flags=flags)
        if ctx.features_only:
            return None, None, None, None, None, gr.features, None, None, None
        return gr.means, gr.log_scales, gr.quats, gr.opacity, gr.colors, gr.features, None, None, None


def render(means: torch.Tensor, log_scales: torch.Tensor, quats: torch.Tensor, opacity: torch.Tensor,
           colors: torch.Tensor, features: torch.Tensor, cam, max_instances: Optional[int] = None,
           features_only: bool = False):
    """Differentiable render of [R, G, B, depth, features...] on the camera's
    sampled grid.  Returns (image [4 + C_sem, H_s, W_s], final_T, n_last);
    only the image carries gradients.  features_only=True propagates to the
    features alone (geometry frozen)."""
    return RenderFunction.apply(means, log_scales, quats, opacity, colors, features, cam, max_instances,
                                features_only)
