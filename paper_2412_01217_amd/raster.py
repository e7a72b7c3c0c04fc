"""Python binding of the C ABI (include/gs.h) on torch tensors.

Argument marshalling only: torch provides device memory and the current stream, and
every step runs in libgs.so's HIP kernels. There is no CPU fallback; without the
built library `_lib.lib()` raises.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as L


def config(n_sem: int, **kw) -> L.Config:
    c = L.Config()
    L.lib().gs_config_default(ctypes.byref(c))
    c.n_sem = int(n_sem)
    for k, v in kw.items():
        if k == "full_rect":
            v = int(v)
        setattr(c, k, v)
    return c


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Frame:
    """The item table of one batch of views: every (view, pyramid level) pair."""

    def __init__(self, cfg: L.Config, views, device="cuda"):
        self.device = torch.device(device)
        self.views = list(views)
        self.tile = (int(cfg.tile_w), int(cfg.tile_h))
        nv = len(views)
        V = (L.View * max(nv, 1))()
        W = (ctypes.c_int32 * max(nv, 1))()
        H = (ctypes.c_int32 * max(nv, 1))()
        K = (ctypes.c_float * max(4 * nv, 1))()
        lv = (ctypes.c_int32 * max(nv, 1))()
        for i, v in enumerate(views):
            R = np.asarray(v.R, np.float32).reshape(9)
            t = np.asarray(v.t, np.float32).reshape(3)
            for k in range(9):
                V[i].R[k] = float(R[k])
            for k in range(3):
                V[i].t[k] = float(t[k])
            W[i], H[i], lv[i] = int(v.W), int(v.H), int(v.levels)
            K[4 * i:4 * i + 4] = [float(v.fx), float(v.fy), float(v.cx), float(v.cy)]
        n_items = sum(int(v.levels) for v in views)
        items = (L.Item * max(n_items, 1))()
        npix = ctypes.c_int64()
        ntile = ctypes.c_int32()
        r = L.lib().gs_make_items(ctypes.byref(cfg), nv, V, W, H, K, lv, items, ctypes.byref(npix), ctypes.byref(ntile))
        if r < 0:
            L.check(r, "gs_make_items")
        self.views_host = V
        self.items = items
        self.n_views = nv
        self.n_items = n_items
        self.n_pixels = int(npix.value)
        self.n_tiles = int(ntile.value)
        self.max_level = max((int(v.levels) - 1 for v in views), default=0)
        self.views_dev = torch.frombuffer(bytearray(bytes(V)), dtype=torch.uint8).to(self.device)
        self.items_dev = torch.frombuffer(bytearray(bytes(items)), dtype=torch.uint8).to(self.device)

    def item_list(self):
        return [dict(W=it.W, H=it.H, view=it.view, level=it.level, tiles_x=it.tiles_x, tiles_y=it.tiles_y,
                     tile_base=it.tile_base, pixel_base=it.pixel_base) for it in self.items[:self.n_items]]


def gaussians_struct(g: dict) -> L.Gaussians:
    s = L.Gaussians()
    s.n = int(g["mean"].shape[0])
    for k in ("mean", "log_scale", "quat", "opacity", "rgb", "sem", "emb"):
        t = g.get(k)
        if t is not None:
            assert t.is_cuda and t.is_contiguous(), k
        setattr(s, k, None if t is None else t.data_ptr())
    return s


def to_device(scene, device="cuda") -> dict:
    d = dict(mean=scene.mean, log_scale=scene.log_scale, quat=scene.quat, opacity=scene.opacity, rgb=scene.rgb)
    out = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(device) for k, v in d.items()}
    if getattr(scene, "sem", None) is not None:
        out["sem"] = torch.as_tensor(np.ascontiguousarray(scene.sem, np.float32)).to(device)
    if getattr(scene, "emb", None) is not None:
        out["emb"] = torch.as_tensor(np.ascontiguousarray(scene.emb).view(np.int16)).to(device)
    return out


def alloc_projected(frame: Frame, n: int) -> dict:
    E = frame.n_items * n
    dev = frame.device
    return dict(rec=torch.empty(E * 8, dtype=torch.float32, device=dev),
                depth=torch.empty(E, dtype=torch.float32, device=dev),
                radius=torch.empty(E, dtype=torch.int32, device=dev))


def preprocess_into(cfg, g: dict, frame: Frame, p: dict) -> dict:
    ps = L.Projected(p["rec"].data_ptr(), p["depth"].data_ptr(), p["radius"].data_ptr())
    gs = gaussians_struct(g)
    L.check(L.lib().gs_preprocess(ctypes.byref(cfg), ctypes.byref(gs), _ptr(frame.views_dev), frame.n_views,
                                  _ptr(frame.items_dev), frame.n_items, ctypes.byref(ps), _stream(frame.device)),
            "gs_preprocess")
    return p


def preprocess(cfg, g: dict, frame: Frame) -> dict:
    return preprocess_into(cfg, g, frame, alloc_projected(frame, int(g["mean"].shape[0])))


def _projected(p: dict) -> L.Projected:
    return L.Projected(p["rec"].data_ptr(), p["depth"].data_ptr(), p["radius"].data_ptr())


def workspace_bytes(kind, cfg, frame, n, capacity=0) -> int:
    b = ctypes.c_size_t()
    L.check(L.lib().gs_workspace_size(kind, ctypes.byref(cfg), frame.n_items, n, frame.n_tiles, capacity,
                                      frame.n_pixels, ctypes.byref(b)), "gs_workspace_size")
    return int(b.value)


class Sorter:
    """Owns the duplicate buffers and the sort workspace for one frame shape."""

    def __init__(self, cfg, frame: Frame, n: int, capacity: int, want_keys=False):
        dev = frame.device
        self.cfg, self.frame, self.n, self.capacity = cfg, frame, n, int(capacity)
        self.ws = torch.empty(workspace_bytes(L.GS_WS_BIN_SORT, cfg, frame, n, self.capacity), dtype=torch.uint8,
                              device=dev)
        self.vals = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.keys = torch.empty(max(self.capacity, 1), dtype=torch.int64, device=dev) if want_keys else None
        self.ranges = torch.empty(2 * max(frame.n_tiles, 1), dtype=torch.int32, device=dev)
        self.n_dup = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)

    def run(self, proj: dict):
        ps = _projected(proj)
        f = self.frame
        L.check(L.lib().gs_bin_sort(ctypes.byref(self.cfg), ctypes.byref(ps), _ptr(f.items_dev), f.n_items, self.n,
                                    f.n_tiles, self.capacity, _ptr(self.ws), self.ws.numel(), _ptr(self.keys),
                                    _ptr(self.vals), _ptr(self.ranges), _ptr(self.n_dup), _ptr(self.status),
                                    _stream(f.device)), "gs_bin_sort")
        return self


def bin_sort(cfg, proj: dict, frame: Frame, n: int, capacity=None, want_keys=False) -> Sorter:
    """Eager binning: grows the capacity (and re-runs) if the duplicates do not fit."""
    cap = int(capacity) if capacity else max(1 << 16, 4 * frame.n_items * n)
    while True:
        s = Sorter(cfg, frame, n, cap, want_keys).run(proj)
        if int(s.status.item()) == L.GS_OK:
            return s
        cap = int(int(s.n_dup.item()) * 1.1) + 1024


def alloc_images(cfg, frame: Frame, n_classes=0, learned=False, state_capacity=None) -> dict:
    """Forward images; with state_capacity (the bin_sort capacity of the lists), also the
    forward state that lets long lists be split and the backward skip its summary pass."""
    K = 4 + cfg.n_sem
    dev = frame.device
    P = frame.n_pixels
    out = dict(color=torch.empty(P * K, dtype=torch.float32, device=dev),
               T=torch.empty(P, dtype=torch.float32, device=dev),
               n_contrib=torch.empty(P, dtype=torch.int32, device=dev), K=K, n_pixels=P)
    out["logits"] = torch.empty(P * n_classes, dtype=torch.float32, device=dev) if learned else None
    out["state"] = None
    if state_capacity is not None:
        nb = workspace_bytes(L.GS_WS_RENDER_STATE, cfg, frame, 0, int(state_capacity))
        out["state"] = torch.empty(nb, dtype=torch.uint8, device=dev)
    return out


def _images(d: dict, P: int = 0) -> L.Images:
    im = L.Images(*(None if d.get(k) is None else d[k].data_ptr() for k in ("color", "T", "n_contrib", "logits")))
    im.n_pixels = int(d.get("n_pixels", P))
    st = d.get("state")
    if st is not None:
        im.state, im.state_bytes = st.data_ptr(), st.numel()
    return im


def head_struct(head: dict | None):
    """head: W1 [64,16] and W2 [C,64] as int16 tensors of bfloat16 bits, b1 [64], b2 [C] float32."""
    if head is None:
        return None
    h = L.Head()
    h.d_in, h.d_hidden, h.n_classes = 16, 64, int(head["b2"].shape[0])
    h.W1, h.b1, h.W2, h.b2 = (head[k].data_ptr() for k in ("W1", "b1", "W2", "b2"))
    return h


def render_fwd(cfg, g: dict, proj: dict, frame: Frame, sorter: Sorter, out=None, head=None, split=True) -> dict:
    """split: allocate the forward state (long lists composited in segments) when out is
    not given; a given out carries its own (or no) state."""
    decode = head is not None
    out = out or alloc_images(cfg, frame, int(head["b2"].shape[0]) if decode else 0, decode,
                              state_capacity=sorter.capacity if split else None)
    gs = gaussians_struct(g)
    ps = _projected(proj)
    im = _images(out, frame.n_pixels)
    hs = head_struct(head)
    L.check(L.lib().gs_render_fwd(ctypes.byref(cfg), ctypes.byref(gs), ctypes.byref(ps), _ptr(frame.items_dev),
                                  frame.n_items, frame.n_tiles, _ptr(sorter.vals), _ptr(sorter.ranges),
                                  ctypes.byref(hs) if hs is not None else None, ctypes.byref(im),
                                  _stream(frame.device)), "gs_render_fwd")
    return out


def loss(cfg, frame: Frame, n_classes: int, rendered: dict, targets: dict, w=(1.0, 1.0, 1.0), grad=None,
         loss_out=None, ws=None, head=None, grads=None, static=False):
    """Per-item loss parts [n_items, 3] and the image gradient. Learned mode with `head`: the
    decode runs inside the loss, grad["color"] channels 4.. receive dL/dE and grads'
    head_W1 .. head_b2 the head's weight gradients (grads: a dict with those four tensors).
    targets["sem_color"] (a 3-channel semantic colour image in the rgb target's layout, with
    cfg.n_sem = 3 and n_classes = 0) selects eq. 12's semantic loss, weighted by
    cfg.sem_ssim_lambda, instead of the cross-entropy on targets["label"].
    static: gs_pyramid_loss_static, whose workspace is the library's own device array."""
    dev = frame.device
    if grad is None:
        grad = dict(color=torch.empty_like(rendered["color"]),
                    logits=(torch.empty_like(rendered["logits"])
                            if rendered.get("logits") is not None and head is None else None))
    loss_out = loss_out if loss_out is not None else torch.empty(3 * frame.n_items, dtype=torch.float32, device=dev)
    if ws is None and not static:
        ws = torch.empty(workspace_bytes(L.GS_WS_LOSS, cfg, frame, 0), dtype=torch.uint8, device=dev)
    t = L.Targets(targets["rgb"].data_ptr(), targets["depth"].data_ptr(),
                  None if targets.get("label") is None else targets["label"].data_ptr(),
                  None if targets.get("sem_color") is None else targets["sem_color"].data_ptr())
    wv = (ctypes.c_float * 3)(*[float(x) for x in w])
    ri = _images(rendered, frame.n_pixels)
    gi = _images(grad, frame.n_pixels)
    hs = head_struct(head)
    gr = None
    if head is not None:
        gr = L.Grads(*(None if grads.get(k) is None else grads[k].data_ptr() for k in GRAD_FIELDS))
    hp = ctypes.byref(hs) if hs is not None else None
    gp = ctypes.byref(gr) if gr is not None else None
    if static:
        L.check(L.lib().gs_pyramid_loss_static(ctypes.byref(cfg), _ptr(frame.items_dev), frame.n_items,
                                               frame.n_pixels, n_classes, ctypes.byref(ri), ctypes.byref(t), hp, wv,
                                               _ptr(loss_out), ctypes.byref(gi), gp, _stream(dev)),
                "gs_pyramid_loss_static")
    else:
        L.check(L.lib().gs_pyramid_loss(ctypes.byref(cfg), _ptr(frame.items_dev), frame.n_items, frame.n_pixels,
                                        n_classes, ctypes.byref(ri), ctypes.byref(t), hp, wv, _ptr(loss_out),
                                        ctypes.byref(gi), gp, _ptr(ws), ws.numel(), _stream(dev)), "gs_pyramid_loss")
    return loss_out.view(frame.n_items, 3), grad


GRAD_FIELDS = ("mean", "log_scale", "quat", "opacity", "rgb", "sem", "emb", "pose", "head_W1", "head_b1", "head_W2",
               "head_b2")


def alloc_grads(cfg, g: dict, frame: Frame, n_classes: int = 0) -> dict:
    n = int(g["mean"].shape[0])
    dev = frame.device
    z = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)  # noqa: E731
    learned = g.get("emb") is not None
    fv = frame.n_views if cfg.view_features else 1        # per-view feature blocks
    out = dict(mean=z(n, 3), log_scale=z(n, 3), quat=z(n, 4), opacity=z(n), rgb=z(fv * n, 3),
               sem=z(fv * n, cfg.n_sem) if (cfg.n_sem and not learned) else None,
               emb=z(n, 16) if learned else None, pose=z(frame.n_views, 6))
    if learned:
        out.update(head_W1=z(64, 16), head_b1=z(64), head_W2=z(n_classes, 64), head_b2=z(n_classes))
    return out


def render_bwd(cfg, g: dict, proj: dict, frame: Frame, sorter: Sorter, fwd: dict, grad_in: dict, grads=None,
               ws=None, head=None) -> dict:
    n = int(g["mean"].shape[0])
    grads = grads or alloc_grads(cfg, g, frame, int(head["b2"].shape[0]) if head is not None else 0)
    if ws is None:
        ws = torch.empty(workspace_bytes(L.GS_WS_RENDER_BWD, cfg, frame, n, sorter.capacity), dtype=torch.uint8,
                         device=frame.device)
    gs = gaussians_struct(g)
    ps = _projected(proj)
    fi = _images(fwd, frame.n_pixels)
    gi = _images(grad_in, frame.n_pixels)
    gr = L.Grads(*(None if grads.get(k) is None else grads[k].data_ptr() for k in GRAD_FIELDS))
    hs = head_struct(head)
    L.check(L.lib().gs_render_bwd(ctypes.byref(cfg), ctypes.byref(gs), ctypes.byref(ps), _ptr(frame.views_dev),
                                  frame.n_views, _ptr(frame.items_dev), frame.n_items, frame.n_tiles,
                                  _ptr(sorter.vals), _ptr(sorter.ranges), ctypes.byref(hs) if hs is not None else None,
                                  ctypes.byref(fi), ctypes.byref(gi), ctypes.byref(gr), _ptr(ws), ws.numel(),
                                  _stream(frame.device)), "gs_render_bwd")
    return grads


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
              bf16_copy: torch.Tensor | None = None, beta1=0.9, beta2=0.999, eps=1e-8):
    L.check(L.lib().gs_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), lr, beta1, beta2, eps,
                                 step, _ptr(bf16_copy), _stream(param.device)), "gs_adam_step")


def sh_struct(sh: dict) -> L.SH:
    """sh: rgb_degree, sem_degree and the band arrays rgb_rest / sem_rest (device)."""
    return L.SH(int(sh.get("rgb_degree", 0)), int(sh.get("sem_degree", 0)), _ptr(sh.get("rgb_rest")),
                _ptr(sh.get("sem_rest")))


def sh_features(g: dict, sh: dict, frame: Frame, out: dict | None = None) -> dict:
    """Per-view features [n_views * n, 3] and [n_views * n, n_sem] of every view of frame,
    for a render with cfg.view_features = 1."""
    n = int(g["mean"].shape[0])
    S = int(g["sem"].shape[1]) if g.get("sem") is not None else 0
    V = frame.n_views
    if out is None:
        out = dict(rgb=torch.empty(V * n, 3, device=frame.device),
                   sem=torch.empty(V * n, S, device=frame.device) if S else None)
    L.check(L.lib().gs_sh_features(S, ctypes.byref(gaussians_struct(g)), ctypes.byref(sh_struct(sh)), _ptr(frame.views_dev), V,
                                   _ptr(out["rgb"]), _ptr(out.get("sem")), _stream(frame.device)), "gs_sh_features")
    return out


def sh_features_bwd(g: dict, sh: dict, frame: Frame, grads: dict, out: dict | None = None) -> dict:
    """Takes gs_render_bwd's per-view feature gradients (grads rgb / sem) to the constant
    bands and SH bands (returned), and adds the direction's share to grads mean and pose."""
    n = int(g["mean"].shape[0])
    S = int(g["sem"].shape[1]) if g.get("sem") is not None else 0
    dev = frame.device
    if out is None:
        z = lambda t: None if t is None else torch.empty_like(t)  # noqa: E731
        out = dict(rgb_dc=torch.empty(n, 3, device=dev), sem_dc=torch.empty(n, S, device=dev) if S else None,
                   rgb_rest=z(sh.get("rgb_rest")), sem_rest=z(sh.get("sem_rest")))
    L.check(L.lib().gs_sh_features_bwd(S, ctypes.byref(gaussians_struct(g)), ctypes.byref(sh_struct(sh)), _ptr(frame.views_dev),
                                       frame.n_views, _ptr(grads["rgb"]), _ptr(grads.get("sem")), _ptr(out["rgb_dc"]),
                                       _ptr(out.get("rgb_rest")), _ptr(out.get("sem_dc")), _ptr(out.get("sem_rest")),
                                       _ptr(grads["mean"]), _ptr(grads["pose"]), _stream(dev)), "gs_sh_features_bwd")
    return out


PARAM_FIELDS = ("mean", "log_scale", "quat", "opacity", "rgb", "sem")


def _param_arrays(d: dict) -> L.ParamArrays:
    return L.ParamArrays(*(None if d.get(k) is None else d[k].data_ptr() for k in PARAM_FIELDS))


def adam_config(lr: dict, beta1=0.9, beta2=0.999, eps=1e-8) -> L.AdamConfig:
    """Learning rates by name (mean, log_scale, quat, opacity, rgb, sem, rho, phi); missing = 0."""
    return L.AdamConfig(*[float(lr.get(k, 0.0)) for k in PARAM_FIELDS + ("rho", "phi")], beta1, beta2, eps)


def gaussians_adam(g: dict, grads: dict, m: dict, v: dict, hp: L.AdamConfig, step: int):
    """One Adam step on every Gaussian parameter group of g (in place), one launch."""
    n = int(g["mean"].shape[0])
    n_sem = int(g["sem"].shape[1]) if g.get("sem") is not None else 0
    gr = L.Grads(*(None if grads.get(k) is None else grads[k].data_ptr() for k in GRAD_FIELDS))
    L.check(L.lib().gs_gaussians_adam(n, n_sem, ctypes.byref(_param_arrays(g)), ctypes.byref(gr),
                                      ctypes.byref(_param_arrays(m)), ctypes.byref(_param_arrays(v)),
                                      ctypes.byref(hp), int(step), _stream(g["mean"].device)), "gs_gaussians_adam")


def pose_adam(views_dev: torch.Tensor, n_views: int, grad_pose: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              hp: L.AdamConfig, step: int):
    """Adam on the pose tangents, then T_cw <- Exp(delta) T_cw of every view in views_dev."""
    L.check(L.lib().gs_pose_adam(_ptr(views_dev), int(n_views), _ptr(grad_pose), _ptr(m), _ptr(v), ctypes.byref(hp),
                                 int(step), _stream(views_dev.device)), "gs_pose_adam")


def pose_perturb(frame: Frame, xi: torch.Tensor, views_out: torch.Tensor | None = None) -> torch.Tensor:
    """The frame's views with T_cw <- Exp(xi_v) T_cw (xi [n_views, 6], device float32),
    as a device gs_view array (views_out, or a new one)."""
    out = views_out if views_out is not None else torch.empty_like(frame.views_dev)
    L.check(L.lib().gs_pose_perturb(_ptr(frame.views_dev), frame.n_views, _ptr(xi), _ptr(out), _stream(frame.device)),
            "gs_pose_perturb")
    return out


def pose_perturb_bwd(xi: torch.Tensor, grad_pose: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dxi from the gradient with respect to a tangent at the perturbed poses."""
    out = out if out is not None else torch.empty_like(grad_pose)
    L.check(L.lib().gs_pose_perturb_bwd(_ptr(xi), int(xi.shape[0]), _ptr(grad_pose), _ptr(out), _stream(xi.device)),
            "gs_pose_perturb_bwd")
    return out


def distill_loss(frame: Frame, C: int, teacher: torch.Tensor, student: torch.Tensor, mse_w=0.1, grad=None,
                 loss_out=None, ws=None):
    dev = frame.device
    grad = grad if grad is not None else torch.empty_like(student)
    loss_out = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=dev)
    ws = ws if ws is not None else torch.empty(256, dtype=torch.uint8, device=dev)
    L.check(L.lib().gs_distill_loss(_ptr(frame.items_dev), frame.n_items, frame.n_pixels, C, _ptr(teacher),
                                    _ptr(student), mse_w, _ptr(loss_out), _ptr(grad), _ptr(ws), ws.numel(),
                                    _stream(dev)), "gs_distill_loss")
    return loss_out, grad


def argmax_agreement(frame: Frame, C: int, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    counts = torch.empty(frame.n_items, dtype=torch.int64, device=frame.device)
    L.check(L.lib().gs_argmax_agreement(_ptr(frame.items_dev), frame.n_items, frame.n_pixels, C, _ptr(a), _ptr(b),
                                        _ptr(counts), _stream(frame.device)), "gs_argmax_agreement")
    return counts


def downsample(frame: Frame, K: int, img: torch.Tensor, labels: torch.Tensor | None = None):
    L.check(L.lib().gs_pyramid_downsample(_ptr(frame.items_dev), frame.n_items, frame.n_pixels, frame.max_level, K,
                                          _ptr(img), _ptr(labels), _stream(frame.device)), "gs_pyramid_downsample")
    return img, labels


class Graph:
    """A captured sequence of library calls (gs_graph_*), replayed on a stream.

    fn() must only enqueue work (every gs_* hot-path call does) on the current torch
    stream, and every buffer it touches must outlive the graph."""

    def __init__(self, fn, device="cuda"):
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.exec = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        with torch.cuda.stream(self.stream):
            s = ctypes.c_void_p(self.stream.cuda_stream)
            L.check(L.lib().gs_graph_begin(s), "gs_graph_begin")
            try:
                fn()
            finally:
                L.check(L.lib().gs_graph_end(s, ctypes.byref(self.exec)), "gs_graph_end")
        torch.cuda.synchronize(self.device)

    def launch(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check(L.lib().gs_graph_launch(self.exec, ctypes.c_void_p(st.cuda_stream)), "gs_graph_launch")

    def __del__(self):
        try:
            if self.exec:
                L.lib().gs_graph_destroy(self.exec)
        except Exception:
            pass
