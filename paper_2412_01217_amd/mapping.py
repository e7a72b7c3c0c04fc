"""Mapping iterations over keyframes with image pyramids (paper Sec. III-C/D).

Each iteration renders a set of (keyframe, pyramid level) items, takes the per-level loss
(eq. 10-13) and back-propagates it to the Gaussians and the keyframe poses; the parameters
then take one Adam step (gs_gaussians_adam, one launch over every group) and each pose
moves by the left-multiplied SE(3) exponential of its Adam step (gs_pose_adam).

Schedules of the items an iteration renders:
  "random"          one (keyframe, level) pair drawn uniformly per iteration, so that every
                    view and every level of the pyramids is trained (Sec. III-C)
  "coarse_to_fine"  the same draw restricted to the coarser levels early on, the resolution
                    rising with training progress: in the first 1/L of the iterations only
                    the coarsest of L levels, then the two coarsest, ..., the last 1/L all
  "batched"         every keyframe at every level in one step (one launch per stage)

Every (keyframe, level) item of the per-pair schedules owns its buffers (a MappingStep
built on first use). Poses live in one device array and are copied into a step's view
table before it runs and back after the update.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import raster, scenes
from .step import MappingStep

# Pose rates default to 0: in the paper's system the mapping thread receives its keyframe
# poses from tracking and bundle adjustment; rho / phi > 0 refines them with the map.
DEFAULT_LR = dict(mean=1e-3, log_scale=5e-3, quat=1e-3, opacity=2.5e-2, rgb=1e-2, sem=1e-2, rho=0.0, phi=0.0)


def render_targets(cfg, frame: raster.Frame, g: dict, device="cuda") -> dict:
    """Target pyramids (eq. 4-6) of every view of `frame`: level 0 rendered from the plain
    scene g, the coarser levels as 2x2 box means of it; labels = argmax of the class
    channels. Planar, in the frame's item layout."""
    K = 4 + cfg.n_sem
    proj = raster.preprocess(cfg, g, frame)
    srt = raster.bin_sort(cfg, proj, frame, int(g["mean"].shape[0]))
    img = raster.render_fwd(cfg, g, proj, frame, srt)
    labels = torch.empty(frame.n_pixels, dtype=torch.int32, device=device)
    raster.downsample(frame, K, img["color"], labels)
    rgb = torch.empty(3 * frame.n_pixels, dtype=torch.float32, device=device)
    depth = torch.empty(frame.n_pixels, dtype=torch.float32, device=device)
    for it in frame.item_list():
        HW, pb = it["W"] * it["H"], it["pixel_base"]
        planes = img["color"][pb * K: pb * K + K * HW].view(K, HW)
        rgb[pb * 3: pb * 3 + 3 * HW] = planes[:3].reshape(-1)
        depth[pb: pb + HW] = planes[3]
    return dict(rgb=rgb, depth=depth, label=labels)


def level_view(v: scenes.View, level: int) -> scenes.View:
    """The single-level view of pyramid level `level` of v (intrinsics and size halved per level)."""
    s = 0.5 ** level
    return scenes.View(v.R, v.t, v.fx * s, v.fy * s, v.cx * s, v.cy * s, v.W >> level, v.H >> level, 1)


@dataclasses.dataclass
class _Unit:
    keyframes: list            # keyframe indices, in the step's view order
    step: MappingStep


class Mapper:
    def __init__(self, cfg, g: dict, keyframes: list, targets: dict, n_classes: int, schedule="random",
                 lr: dict | None = None, w=(1.0, 1.0, 1.0), fixed_poses=(0,), iterations=1000, seed=0,
                 beta1=0.9, beta2=0.999, eps=1e-15):
        """cfg: library config (n_sem = n_classes, plain semantics); g: the Gaussians (device,
        updated in place); keyframes: views with `levels` pyramid levels each; targets: the
        pyramids of all keyframes in raster.Frame(cfg, keyframes) layout (render_targets);
        fixed_poses: keyframes whose pose is not optimised; iterations: the schedule's length
        (coarse_to_fine uses it for its progress)."""
        if schedule not in ("random", "coarse_to_fine", "batched"):
            raise ValueError(schedule)
        self.cfg, self.g, self.n_classes, self.schedule = cfg, g, n_classes, schedule
        self.w = tuple(float(x) for x in w)
        self.keyframes = list(keyframes)
        self.levels = int(keyframes[0].levels)
        if any(int(v.levels) != self.levels for v in keyframes):
            raise ValueError("every keyframe needs the same number of pyramid levels")
        self.dev = g["mean"].device
        self.all = raster.Frame(cfg, keyframes, device=self.dev)
        self.targets = targets
        self.items = self.all.item_list()
        self.iterations = int(iterations)
        self.rng = np.random.default_rng(seed)
        lr = dict(DEFAULT_LR if lr is None else lr)
        self.hp = raster.adam_config(lr, beta1, beta2, eps)
        self.pose_hp = raster.adam_config({k: lr.get(k, 0.0) for k in ("rho", "phi")}, beta1, beta2, eps)
        self.fixed = set(int(k) for k in fixed_poses)
        nk = len(keyframes)
        self.poses = torch.tensor(np.stack([np.concatenate([np.asarray(v.R, np.float32).reshape(9),
                                                            np.asarray(v.t, np.float32).reshape(3)])
                                            for v in keyframes]), dtype=torch.float32, device=self.dev)
        self.pose_m = torch.zeros(nk, 6, device=self.dev)
        self.pose_v = torch.zeros(nk, 6, device=self.dev)
        self.pose_steps = [0] * nk
        self.m = {k: torch.zeros_like(t) for k, t in g.items() if k in raster.PARAM_FIELDS and t is not None}
        self.v = {k: torch.zeros_like(t) for k, t in g.items() if k in raster.PARAM_FIELDS and t is not None}
        self.step_count = 0
        self.units: dict = {}

    # ------------------------------------------------------------------ items
    def _unit(self, key) -> _Unit:
        u = self.units.get(key)
        if u is None:
            u = self._build(key)
            self.units[key] = u
        return u

    def _build(self, key) -> _Unit:
        cfg = self.cfg
        if key == "all":
            fr, kfs, tg = self.all, list(range(len(self.keyframes))), self.targets
        else:
            k, l = key
            fr = raster.Frame(cfg, [level_view(self.keyframes[k], l)], device=self.dev)
            it = self.items[k * self.levels + l]
            HW, pb = it["W"] * it["H"], it["pixel_base"]
            tg = dict(rgb=self.targets["rgb"][3 * pb: 3 * pb + 3 * HW].contiguous(),
                      depth=self.targets["depth"][pb: pb + HW].contiguous(),
                      label=self.targets["label"][pb: pb + HW].contiguous())
            kfs = [k]
        self._load_poses(fr, kfs)
        return _Unit(kfs, MappingStep(cfg, fr, self.g, tg, self.n_classes, w=self.w, split=True))

    def _load_poses(self, fr: raster.Frame, kfs):
        vf = fr.views_dev.view(torch.float32).view(-1, 14)
        vf[:, :12] = self.poses[kfs]

    def _store_poses(self, fr: raster.Frame, kfs):
        vf = fr.views_dev.view(torch.float32).view(-1, 14)
        self.poses[kfs] = vf[:, :12]

    def draw(self, i: int):
        """The item set of iteration i: "all", or a (keyframe, level) pair."""
        if self.schedule == "batched":
            return "all"
        L = self.levels
        lo = 0
        if self.schedule == "coarse_to_fine":
            stage = min(L - 1, (i * L) // max(self.iterations, 1))
            lo = L - 1 - stage                     # finest level allowed so far
        k = int(self.rng.integers(len(self.keyframes)))
        lvl = int(self.rng.integers(lo, L))
        return (k, lvl)

    # ------------------------------------------------------------------ one iteration
    def iteration(self, i: int | None = None, check_capacity=True) -> dict:
        """Render, loss, backward and update for the item set of iteration i (default: the
        next one). Returns {"key", "loss" (device [n_items, 3])}. check_capacity reads the
        bin sort's status back and rebuilds an item whose duplicates outgrew its buffers."""
        i = self.step_count if i is None else i
        key = self.draw(i)
        u = self._unit(key)
        st = u.step
        self._load_poses(st.frame, u.keyframes)
        st.run()
        if check_capacity and st.overflowed():
            self.units.pop(key)
            u = self._unit(key)
            st = u.step
            st.run()
            if st.overflowed():
                raise RuntimeError("duplicate capacity exceeded after a rebuild")
        self.step_count += 1
        raster.gaussians_adam(self.g, st.grads, self.m, self.v, self.hp, self.step_count)
        live = [j for j, k in enumerate(u.keyframes) if k not in self.fixed]
        if live and (self.pose_hp.lr_rho != 0.0 or self.pose_hp.lr_phi != 0.0):
            for j in live:
                k = u.keyframes[j]
                self.pose_steps[k] += 1
                row = st.frame.views_dev[56 * j: 56 * (j + 1)]
                raster.pose_adam(row, 1, st.grads["pose"][j], self.pose_m[k], self.pose_v[k], self.pose_hp,
                                 self.pose_steps[k])
            self._store_poses(st.frame, u.keyframes)
        return dict(key=key, loss=st.loss.view(-1, 3))

    def total_loss(self, key) -> float:
        """w . loss summed over the items of the last run of `key` (reads back)."""
        st = self.units[key].step
        return float((st.loss.view(-1, 3) * torch.tensor(self.w, device=self.dev)).sum().item())

    def evaluate(self) -> float:
        """Weighted loss over every keyframe and level at the current parameters (no update;
        runs the batched step, whose gradients are discarded)."""
        u = self._unit("all")
        self._load_poses(u.step.frame, u.keyframes)
        u.step.run()
        return self.total_loss("all")
