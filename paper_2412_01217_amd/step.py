"""One mapping iteration of the pyramid rasterizer (paper Sec. III-C/D) with every
buffer allocated up front, so that it can be replayed eagerly or as a HIP graph.

run(): projection -> binning -> compositing -> per-level loss -> backward, all items
       of the frame, through the C ABI on the current torch stream. With a head
       (learned mode) the loss's semantic term acts on the decoded logits: by default the
       decode, its cross-entropy and the decode's backward run inside the loss call
       (fused_head), so no logits are stored; fused_head=False decodes in the forward and
       differentiates the head in the backward instead. With SH bands
       (`sh`), the per-view features are evaluated after the projection and the backward
       ends with their gradients (to the bands in `sh_grads`, to means and poses in place).
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import raster


class MappingStep:
    def __init__(self, cfg, frame: raster.Frame, g: dict, targets: dict, n_classes: int, w=(1.0, 1.0, 1.0),
                 capacity_margin=1.15, head: dict | None = None, split=True, sh: dict | None = None,
                 fused_head=True):
        if sh is not None and not cfg.view_features:
            raise ValueError("SH features need a config with view_features = 1")
        self.cfg, self.frame, self.g, self.targets = cfg, frame, g, targets
        self.sh = sh
        self.feats = raster.sh_features(g, sh, frame) if sh is not None else None
        self.sh_grads = None
        # the render reads the per-view feature blocks in place of the constant bands
        self.g_render = dict(g, rgb=self.feats["rgb"], sem=self.feats["sem"]) if sh is not None else g
        self.n_classes = n_classes
        self.head = head
        self.w = tuple(float(x) for x in w)
        dev = frame.device
        n = int(g["mean"].shape[0])
        self.n = n
        self.proj = raster.preprocess(cfg, g, frame)
        probe = raster.bin_sort(cfg, self.proj, frame, n)
        self.n_dup_probe = int(probe.n_dup.item())
        self.n_visible_probe = int((self.proj["radius"] > 0).sum().item())
        del probe
        self.sorter = raster.Sorter(cfg, frame, n, capacity=int(self.n_dup_probe * capacity_margin) + 4096)
        learned = head is not None
        self.fused_head = learned and fused_head
        decode = learned and not self.fused_head          # logits stored between the calls
        self.img = raster.alloc_images(cfg, frame, n_classes if decode else 0, decode,
                                       state_capacity=self.sorter.capacity if split else None)
        self.grad = dict(color=torch.zeros_like(self.img["color"]),
                         logits=torch.empty_like(self.img["logits"]) if decode else None)
        self.loss = torch.empty(3 * frame.n_items, dtype=torch.float32, device=dev)
        self.loss_ws = torch.empty(raster.workspace_bytes(L.GS_WS_LOSS, cfg, frame, n), dtype=torch.uint8,
                                   device=dev)
        self.grads = raster.alloc_grads(cfg, g, frame, n_classes)
        if sh is not None:
            z = lambda t: None if t is None else torch.empty_like(t)  # noqa: E731
            S = cfg.n_sem
            self.sh_grads = dict(rgb_dc=torch.empty(n, 3, device=dev),
                                 sem_dc=torch.empty(n, S, device=dev) if S else None,
                                 rgb_rest=z(sh.get("rgb_rest")), sem_rest=z(sh.get("sem_rest")))
        self.bwd_ws = torch.empty(raster.workspace_bytes(L.GS_WS_RENDER_BWD, cfg, frame, n, self.sorter.capacity),
                                  dtype=torch.uint8,
                                  device=dev)

    def run(self, ev=None):
        """Enqueue one step. ev: optional list of 5 torch events recorded between the calls."""
        cfg, fr, g = self.cfg, self.frame, self.g
        raster.preprocess_into(cfg, g, fr, self.proj)
        if self.sh is not None:
            raster.sh_features(g, self.sh, fr, out=self.feats)
        gr = self.g_render
        if ev:
            ev[0].record()
        self.sorter.run(self.proj)
        if ev:
            ev[1].record()
        fused = self.fused_head
        raster.render_fwd(cfg, gr, self.proj, fr, self.sorter, out=self.img, head=None if fused else self.head)
        if ev:
            ev[2].record()
        raster.loss(cfg, fr, self.n_classes, self.img, self.targets, w=self.w, grad=self.grad, loss_out=self.loss,
                    ws=self.loss_ws, head=self.head if fused else None, grads=self.grads)
        if ev:
            ev[3].record()
        raster.render_bwd(cfg, gr, self.proj, fr, self.sorter, self.img, self.grad, grads=self.grads, ws=self.bwd_ws,
                          head=None if fused else self.head)
        if self.sh is not None:
            raster.sh_features_bwd(g, self.sh, fr, self.grads, out=self.sh_grads)
        if ev:
            ev[4].record()

    def capture(self) -> raster.Graph:
        return raster.Graph(self.run, self.frame.device)

    def overflowed(self) -> bool:
        return int(self.sorter.status.item()) != L.GS_OK
