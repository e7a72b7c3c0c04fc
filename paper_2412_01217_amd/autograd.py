"""torch.autograd.Function around the rasterizer (paper Sec. III-C/D).

forward:  projection -> binning -> compositing of every item of a Frame, returning
          the planar image [P * (4 + n_sem)] (rgb, depth, semantic channels per item).
backward: gs_render_bwd, returning gradients for every Gaussian parameter and for a
          per-view pose tangent xi = (rho, phi) of T_cw <- Exp(xi) T_cw.

The pose enters as a tangent at the frame's stored poses: pass a zero tensor
[n_views, 6] with requires_grad to receive dL/dxi at xi = 0. Both passes run in the
HIP library; torch only supplies memory and the stream.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import raster


class RenderPyramid(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, rgb, sem, pose_xi, frame, cfg, capacity=None):
        g = dict(mean=mean.contiguous(), log_scale=log_scale.contiguous(), quat=quat.contiguous(),
                 opacity=opacity.contiguous(), rgb=rgb.contiguous(), sem=sem.contiguous() if sem is not None else None)
        n = int(mean.shape[0])
        proj = raster.preprocess(cfg, g, frame)
        sorter = raster.bin_sort(cfg, proj, frame, n, capacity=capacity)
        img = raster.render_fwd(cfg, g, proj, frame, sorter)
        ctx.state = (g, proj, sorter, img, frame, cfg)
        ctx.mark_non_differentiable(img["T"], img["n_contrib"])
        return img["color"], img["T"], img["n_contrib"]

    @staticmethod
    def backward(ctx, gcolor, _gT, _gnc):
        g, proj, sorter, img, frame, cfg = ctx.state
        grads = raster.render_bwd(cfg, g, proj, frame, sorter, img, dict(color=gcolor.contiguous(), logits=None))
        ctx.state = None
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity"], grads["rgb"], grads["sem"],
                grads["pose"], None, None, None)


def render(params: dict, frame: raster.Frame, cfg: L.Config, pose_xi: torch.Tensor | None = None, capacity=None):
    """Differentiable render of every item of `frame`. params: mean, log_scale, quat,
    opacity, rgb, sem (torch CUDA tensors). Returns (color, T, n_contrib)."""
    if pose_xi is None:
        pose_xi = torch.zeros(frame.n_views, 6, device=frame.device)
    return RenderPyramid.apply(params["mean"], params["log_scale"], params["quat"], params["opacity"], params["rgb"],
                               params.get("sem"), pose_xi, frame, cfg, capacity)
