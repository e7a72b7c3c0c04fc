"""Learned semantic head: fitting per-Gaussian 16-dim embeddings and the 16->64->C
MLP so that decoded logits reproduce the plain C-class render (the paper composites
semantic features directly, eq. 9; the learned form replaces the C-wide feature by a
16-wide embedding plus a per-pixel decoder).

Training objective (a reading, the paper has no learned head): soft-target
cross-entropy of the decoded logits against the plain render plus 0.1 times their
mean squared difference; Adam, lr 3e-3 for the MLP and 3e-2 for the embeddings, both
decayed to 0 by a half cosine over the steps; one random view (with its pyramid) per step, either drawn from a fixed pool or generated
fresh for every step so that every Gaussian is eventually seen. Forward, backward,
loss and optimizer all run in the library's kernels; geometry is held fixed, so a
pooled view's projection and binning are computed once.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import raster, scenes


class Head:
    """Float32 master weights, bfloat16 copies used by the kernels, Adam moments."""

    def __init__(self, n_classes: int, device="cuda", seed=6000):
        w = scenes.head_weights(n_classes, seed)
        dev = torch.device(device)
        self.C = n_classes
        self.W1 = torch.from_numpy(w["W1"].view(np.int16).copy()).to(dev)
        self.W2 = torch.from_numpy(w["W2"].view(np.int16).copy()).to(dev)
        self.b1 = torch.from_numpy(w["b1"]).to(dev)
        self.b2 = torch.from_numpy(w["b2"]).to(dev)
        self.W1_master = torch.from_numpy(scenes.bf16_bits_to_f32(w["W1"]).copy()).to(dev)
        self.W2_master = torch.from_numpy(scenes.bf16_bits_to_f32(w["W2"]).copy()).to(dev)
        self.moments = {k: (torch.zeros_like(t), torch.zeros_like(t))
                        for k, t in (("W1", self.W1_master), ("W2", self.W2_master), ("b1", self.b1), ("b2", self.b2))}

    def as_dict(self):
        return dict(W1=self.W1, b1=self.b1, W2=self.W2, b2=self.b2)

    def step(self, grads: dict, lr: float, t: int):
        for k, master, bf in (("W1", self.W1_master, self.W1), ("W2", self.W2_master, self.W2)):
            m, v = self.moments[k]
            raster.adam_step(master, grads["head_" + k], m, v, lr, t, bf16_copy=bf)
        for k, p in (("b1", self.b1), ("b2", self.b2)):
            m, v = self.moments[k]
            raster.adam_step(p, grads["head_" + k], m, v, lr, t)


class ViewState:
    """One view (with its pyramid): frame, fixed projection and binning, buffers."""

    def __init__(self, cfg_plain, cfg_learned, view, g_plain, g_learned, n, C, head, device):
        self.fr = raster.Frame(cfg_learned, [view], device=device)
        fr_plain = raster.Frame(cfg_plain, [view], device=device)
        proj = raster.preprocess(cfg_plain, g_plain, fr_plain)
        self.sorter = raster.bin_sort(cfg_plain, proj, fr_plain, n)
        self.proj = proj
        plain = raster.render_fwd(cfg_plain, g_plain, proj, fr_plain, self.sorter)
        # the plain render's class logits (channels 4..) in a C-plane layout per item
        K = 4 + C
        self.teacher = torch.empty(fr_plain.n_pixels * C, dtype=torch.float32, device=device)
        for it in fr_plain.item_list():
            HW = it["W"] * it["H"]
            pb = it["pixel_base"]
            self.teacher[pb * C: pb * C + C * HW] = plain["color"][pb * K + 4 * HW: pb * K + K * HW]
        del plain
        self.img = raster.alloc_images(cfg_learned, self.fr, C, learned=True, state_capacity=self.sorter.capacity)
        self.grad = dict(color=torch.zeros_like(self.img["color"]), logits=torch.empty_like(self.img["logits"]))
        self.grads = raster.alloc_grads(cfg_learned, g_learned, self.fr, C)
        self.ws = torch.empty(raster.workspace_bytes(raster.L.GS_WS_RENDER_BWD, cfg_learned, self.fr, n,
                                                     self.sorter.capacity),
                              dtype=torch.uint8, device=device)
        self.loss = torch.empty(1, dtype=torch.float32, device=device)
        self.dws = torch.empty(256, dtype=torch.uint8, device=device)


class Trainer:
    """views: a list (a pool, one drawn at random per step) or a callable step -> View
    (a fresh view per step)."""

    def __init__(self, scene, views, n_classes: int, device="cuda", seed=6000):
        self.device = torch.device(device)
        self.C = n_classes
        self.cfg_plain = raster.config(n_classes)
        self.cfg_learned = raster.config(16)
        g = raster.to_device(scene, device)
        self.g_plain = {k: v for k, v in g.items() if k != "emb"}
        self.emb_master = torch.from_numpy(scenes.bf16_bits_to_f32(scene.emb).copy()).to(self.device)
        self.emb_m = torch.zeros_like(self.emb_master)
        self.emb_v = torch.zeros_like(self.emb_master)
        self.g_learned = {k: v for k, v in g.items() if k != "sem"}
        self.head = Head(n_classes, device, seed)
        self.n = scene.n
        self.view_fn = views if callable(views) else None
        self.views = [] if callable(views) else [self._state(v) for v in views]
        self.rng = np.random.default_rng(seed)
        self.t = 0

    def _state(self, view) -> ViewState:
        return ViewState(self.cfg_plain, self.cfg_learned, view, self.g_plain, self.g_learned, self.n, self.C,
                         self.head, self.device)

    def forward(self, vs: ViewState):
        raster.render_fwd(self.cfg_learned, self.g_learned, vs.proj, vs.fr, vs.sorter, out=vs.img,
                          head=self.head.as_dict())

    def train(self, steps: int, lr_mlp=3e-3, lr_emb=3e-2, mse_w=0.1, schedule="cosine"):
        """schedule: "constant" rates, or "cosine" (each rate times (1 + cos(pi k / steps)) / 2
        at step k, decaying to 0 at the end)."""
        losses = []
        for k in range(steps):
            f = 1.0 if schedule == "constant" else 0.5 * (1.0 + math.cos(math.pi * k / steps))
            if self.view_fn is not None:
                vs = self._state(self.view_fn(self.t))
            else:
                vs = self.views[int(self.rng.integers(len(self.views)))]
            self.forward(vs)
            vs.grad["color"].zero_()      # the head's backward adds to the embedding channels
            raster.distill_loss(vs.fr, self.C, vs.teacher, vs.img["logits"], mse_w, grad=vs.grad["logits"],
                                loss_out=vs.loss, ws=vs.dws)
            raster.render_bwd(self.cfg_learned, self.g_learned, vs.proj, vs.fr, vs.sorter, vs.img, vs.grad,
                              grads=vs.grads, ws=vs.ws, head=self.head.as_dict())
            self.t += 1
            raster.adam_step(self.emb_master, vs.grads["emb"], self.emb_m, self.emb_v, lr_emb * f, self.t,
                             bf16_copy=self.g_learned["emb"])
            self.head.step(vs.grads, lr_mlp * f, self.t)
            losses.append(vs.loss)
        return torch.stack([x.clone() for x in losses[-10:]]).mean().item() if losses else float("nan")

    def evaluate(self, views) -> dict:
        """Argmax agreement and logit error of the decoded logits against the plain render."""
        agree = total = 0
        se = n = 0.0
        for v in views:
            vs = self._state(v)
            self.forward(vs)
            counts = raster.argmax_agreement(vs.fr, self.C, vs.teacher, vs.img["logits"])
            agree += int(counts.sum().item())
            total += vs.fr.n_pixels
            d = vs.img["logits"] - vs.teacher
            se += float((d * d).sum().item())
            n += d.numel()
        return dict(agreement=agree / max(total, 1), logit_rmse=(se / max(n, 1)) ** 0.5, pixels=total)
