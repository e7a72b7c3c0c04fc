"""torch.autograd.Function around the rasterizer (paper Sec. III-C/D).

forward:  pose perturbation -> projection -> binning -> compositing of every item of a
          Frame, returning the planar image [P * (4 + n_sem)] (rgb, depth, semantic
          channels per item) and, with a learned head, the decoded logits [P * C].
backward: gs_render_bwd, returning gradients for every Gaussian parameter (the class
          logits, or the embedding), the head's weights, and the per-view pose tangent.

The pose enters as a left perturbation xi = (rho, phi) of each view's stored pose,
T_cw <- Exp(xi) T_cw (gs_pose_perturb); its gradient at any xi is the library's tangent
gradient at the perturbed pose taken through SE(3)'s left Jacobian (gs_pose_perturb_bwd).
Pass zeros [n_views, 6] with requires_grad for dL/dxi at the stored poses.

Learned mode: the embedding [n, 16] and the head's W1 [64, 16], W2 [C, 64] are float32
tensors whose values the kernels read rounded to bfloat16 (the stored precision); their
gradients are those of the rounded values (exact when the values are bfloat16 already, as
with a float32 master copy kept in step with its bfloat16 copy). b1 [64], b2 [C] are float32.
Every pass runs in the HIP library; torch only supplies memory and the stream.
"""
from __future__ import annotations

import copy

import torch

from . import _lib as L
from . import raster


def _bf16_bits(t: torch.Tensor) -> torch.Tensor:
    return t.detach().to(torch.bfloat16).contiguous().view(torch.int16)


class RenderPyramid(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, rgb, sem, emb, W1, b1, W2, b2, pose_xi, frame, cfg,
                capacity=None):
        learned = emb is not None
        g = dict(mean=mean.detach().contiguous(), log_scale=log_scale.detach().contiguous(),
                 quat=quat.detach().contiguous(), opacity=opacity.detach().contiguous(), rgb=rgb.detach().contiguous())
        head = None
        if learned:
            g["emb"] = _bf16_bits(emb)
            head = dict(W1=_bf16_bits(W1), b1=b1.detach().float().contiguous(), W2=_bf16_bits(W2),
                        b2=b2.detach().float().contiguous())
        else:
            g["sem"] = sem.detach().contiguous() if sem is not None else None
        xi = pose_xi.detach().float().contiguous()
        fr = copy.copy(frame)
        fr.views_dev = raster.pose_perturb(frame, xi)
        n = int(mean.shape[0])
        proj = raster.preprocess(cfg, g, fr)
        sorter = raster.bin_sort(cfg, proj, fr, n, capacity=capacity)
        img = raster.render_fwd(cfg, g, proj, fr, sorter, head=head)
        logits = img["logits"] if learned else torch.empty(0, device=mean.device)
        ctx.state = (g, head, xi, proj, sorter, img, fr, cfg)
        ctx.mark_non_differentiable(img["T"], img["n_contrib"])
        if not learned:
            ctx.mark_non_differentiable(logits)
        return img["color"], logits, img["T"], img["n_contrib"]

    @staticmethod
    def backward(ctx, gcolor, glogits, _gT, _gnc):
        g, head, xi, proj, sorter, img, fr, cfg = ctx.state
        learned = head is not None
        gin = dict(color=gcolor.contiguous().clone() if learned else gcolor.contiguous(), logits=None)
        if learned:
            # the library overwrites the embedding channels of the colour gradient with the
            # head's input gradient, so it gets a copy
            gin["logits"] = glogits.contiguous() if glogits is not None else torch.zeros_like(img["logits"])
        grads = raster.render_bwd(cfg, g, proj, fr, sorter, img, gin, head=head)
        gxi = raster.pose_perturb_bwd(xi, grads["pose"])
        ctx.state = None
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity"], grads["rgb"], grads.get("sem"),
                grads.get("emb"), grads.get("head_W1"), grads.get("head_b1"), grads.get("head_W2"),
                grads.get("head_b2"), gxi, None, None, None)


def _xi(frame, pose_xi):
    return torch.zeros(frame.n_views, 6, device=frame.device) if pose_xi is None else pose_xi


def render(params: dict, frame: raster.Frame, cfg: L.Config, pose_xi: torch.Tensor | None = None, capacity=None):
    """Differentiable render of every item of `frame`. params: mean, log_scale, quat,
    opacity, rgb, sem (torch CUDA tensors). Returns (color, T, n_contrib)."""
    color, _, T, nc = RenderPyramid.apply(params["mean"], params["log_scale"], params["quat"], params["opacity"],
                                          params["rgb"], params.get("sem"), None, None, None, None, None,
                                          _xi(frame, pose_xi), frame, cfg, capacity)
    return color, T, nc


def render_learned(params: dict, head: dict, frame: raster.Frame, cfg: L.Config, pose_xi: torch.Tensor | None = None,
                   capacity=None):
    """Differentiable render with the learned semantic head. params: mean, log_scale, quat,
    opacity, rgb and emb [n, 16] (float32); head: W1 [64, 16], b1 [64], W2 [C, 64], b2 [C]
    (float32); cfg.n_sem = 16. Returns (color [P * 20], logits [P * C], T, n_contrib)."""
    return RenderPyramid.apply(params["mean"], params["log_scale"], params["quat"], params["opacity"], params["rgb"],
                               None, params["emb"], head["W1"], head["b1"], head["W2"], head["b2"],
                               _xi(frame, pose_xi), frame, cfg, capacity)
