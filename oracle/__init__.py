"""Test infrastructure: Python access to the FP64 CPU oracle in gs_oracle.cpp.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package. It never imports the HIP library or the package around it; it reads plain
numpy arrays (any object with the attribute names below works as a scene or view).

Every function converts its inputs to float64 before calling the C++ oracle, which
runs single-threaded in double precision.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no threads, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_sort_stage.restype = ctypes.c_int64
        _lib.or_distill.restype = ctypes.c_double
        _lib.or_distill.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    return _lib


@dataclasses.dataclass
class Config:
    tile_w: int = 16
    tile_h: int = 16
    z_near: float = 0.2
    eps: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    guard: float = 1.3
    full_rect: bool = False
    # Relative closeness to a threshold that flags a per-pixel decision (alpha_min, alpha_max,
    # t_min). It bounds the single-precision path's relative error at the decision: alpha
    # carries the rounding of the pixel offset and the exponent (a few 1e-6), and T after n
    # blends carries up to about n * 1.5 ulp (n * 9e-8), which for the 100-200 blends before a
    # t_min stop in the room workloads is 1e-5 to 2e-5.
    margin: float = 2e-5
    margin_pre: float = 1e-9    # projection decisions (z_near, guard, radius and rect rounding)
    isotropic: bool = False     # the primitive of eq. 1-3: one scale (log_scale[:, 0]), no rotation

    def exact(self) -> "Config":
        """Cut-offs removed: every Gaussian covers every tile, no alpha_min / t_min."""
        return dataclasses.replace(self, alpha_min=0.0, t_min=0.0, full_rect=True)

    def arrays(self, S: int):
        cd = np.array([self.z_near, self.eps, self.alpha_min, self.alpha_max, self.t_min,
                       self.guard, self.margin, self.margin_pre], np.float64)
        ci = np.array([self.tile_w, self.tile_h, int(self.full_rect), S, int(self.isotropic)], np.int32)
        return cd, ci


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _views(views):
    vd = np.zeros((len(views), 16), np.float64)
    vi = np.zeros((len(views), 3), np.int32)
    for k, v in enumerate(views):
        vd[k, :9] = np.asarray(v.R, np.float64).reshape(9)
        vd[k, 9:12] = np.asarray(v.t, np.float64)
        vd[k, 12:16] = [v.fx, v.fy, v.cx, v.cy]
        vi[k] = [v.W, v.H, v.levels]
    return vd, vi


def items(views, tile_w=16, tile_h=16):
    """The (view, level) items in order, with sizes and offsets."""
    out = []
    pix = 0
    tile = 0
    for v_i, v in enumerate(views):
        for l in range(v.levels):
            W, H = v.W >> l, v.H >> l
            ntx, nty = -(-W // tile_w), -(-H // tile_h)
            out.append(dict(view=v_i, level=l, W=W, H=H, ntx=ntx, nty=nty, tile0=tile, pix0=pix))
            pix += W * H
            tile += ntx * nty
    return out


def layout(views, tile_w=16, tile_h=16):
    it = items(views, tile_w, tile_h)
    return len(it), sum(i["W"] * i["H"] for i in it), sum(i["ntx"] * i["nty"] for i in it)


def _gauss(scene, sem):
    sem = scene.sem if sem is None else sem
    S = 0 if sem is None else int(np.asarray(sem).shape[1])
    g = [_d(scene.mean), _d(scene.log_scale), _d(scene.quat), _d(scene.opacity), _d(scene.rgb),
         _d(sem) if S else np.zeros((scene.mean.shape[0], 0))]
    return g, S


def preprocess(cfg: Config, scene, views):
    lib = _load()
    n = scene.mean.shape[0]
    n_items, _, _ = layout(views, cfg.tile_w, cfg.tile_h)
    cd, ci = cfg.arrays(0)
    vd, vi = _views(views)
    E = n_items * n
    out = dict(m2=np.zeros((E, 2)), conic=np.zeros((E, 3)), opacity=np.zeros(E), depth=np.zeros(E),
               radius=np.zeros(E, np.int32), rect=np.zeros((E, 4), np.int32), flag=np.zeros(E, np.int32))
    g, _ = _gauss(scene, np.zeros((n, 0)))
    lib.or_preprocess(_p(cd), _p(ci), ctypes.c_int64(n), _p(g[0]), _p(g[1]), _p(g[2]), _p(g[3]),
                      ctypes.c_int(len(views)), _p(vd), _p(vi), _p(out["m2"]), _p(out["conic"]),
                      _p(out["opacity"]), _p(out["depth"]), _p(out["radius"]), _p(out["rect"]),
                      _p(out["flag"]))
    return out


def render(cfg: Config, scene, views, sem=None, brute=False, tile_mask=None):
    """Images [P*K] planar per item, T [P], n_contrib [P], flag [P] (near-threshold pixels)."""
    lib = _load()
    n = scene.mean.shape[0]
    g, S = _gauss(scene, sem)
    K = 4 + S
    _, P, T = layout(views, cfg.tile_w, cfg.tile_h)
    cd, ci = cfg.arrays(S)
    vd, vi = _views(views)
    img = np.zeros(P * K)
    Tout = np.zeros(P)
    nc = np.zeros(P, np.int32)
    fl = np.zeros(P, np.int32)
    nb = np.zeros(P, np.int32)
    mask = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    lib.or_render(_p(cd), _p(ci), ctypes.c_int64(n), *[_p(a) for a in g], ctypes.c_int(len(views)), _p(vd),
                  _p(vi), ctypes.c_int(int(brute)), _p(mask), _p(img), _p(Tout), _p(nc), _p(fl), _p(nb))
    return dict(img=img, T=Tout, n_contrib=nc, flag=fl, n_blend=nb, K=K)


def backward(cfg: Config, scene, views, gimg, sem=None, tile_mask=None, want_g2d=False):
    """Gradient of sum(gimg * render(...)['img']) with respect to every input; with
    want_g2d also the per (item, Gaussian) 2D gradients [n_items * n, 7]."""
    lib = _load()
    n = scene.mean.shape[0]
    g, S = _gauss(scene, sem)
    n_items, P, _ = layout(views, cfg.tile_w, cfg.tile_h)
    cd, ci = cfg.arrays(S)
    vd, vi = _views(views)
    out = dict(mean=np.zeros((n, 3)), log_scale=np.zeros((n, 3)), quat=np.zeros((n, 4)),
               opacity=np.zeros(n), rgb=np.zeros((n, 3)), sem=np.zeros((n, S)),
               pose=np.zeros((len(views), 6)), g2d=np.zeros((n_items * n, 7)) if want_g2d else None,
               gflag=np.zeros(n, np.int32))
    gimg = _d(gimg)
    mask = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    lib.or_backward(_p(cd), _p(ci), ctypes.c_int64(n), *[_p(a) for a in g], ctypes.c_int(len(views)), _p(vd),
                    _p(vi), _p(mask), _p(gimg), _p(out["mean"]), _p(out["log_scale"]), _p(out["quat"]),
                    _p(out["opacity"]), _p(out["rgb"]), _p(out["sem"]), _p(out["pose"]), _p(out["g2d"]),
                    _p(out["gflag"]))
    return out


def loss(views, S, img, t_rgb, t_depth, t_label, w=(1.0, 1.0, 1.0), tile_w=16, tile_h=16, ssim_lambda=0.0,
         t_sem=None, sem_ssim_lambda=0.0):
    """Per-item [L_rgb, L1 depth (valid), L_sem] and the image-layout gradient of
    w . sum over items. L_rgb = (1 - lambda) mean L1 + lambda (1 - mean SSIM); lambda = 0
    gives the plain L1 mean. L_sem is the cross-entropy against t_label, or, with t_sem (a
    3-channel semantic colour image in the t_rgb layout, S = 3), eq. 12: the same form as
    L_rgb on the semantic channels with lambda = sem_ssim_lambda."""
    lib = _load()
    if t_sem is not None and S != 3:
        raise ValueError("the semantic colour loss composites 3 semantic channels")
    n_items, P, _ = layout(views, tile_w, tile_h)
    K = 4 + S
    _, ci = Config(tile_w=tile_w, tile_h=tile_h).arrays(S)
    vi = _views(views)[1]
    ls = np.zeros((n_items, 3))
    gimg = np.zeros(P * K)
    lab = np.ascontiguousarray(np.zeros(P, np.int32) if t_label is None else t_label, dtype=np.int32)
    w5 = np.array([w[0], w[1], w[2], ssim_lambda, sem_ssim_lambda], np.float64)
    ts = None if t_sem is None else _d(t_sem)
    rc = lib.or_loss(_p(ci), ctypes.c_int(len(views)), _p(vi), _p(_d(img)), _p(_d(t_rgb)), _p(_d(t_depth)),
                     _p(lab), _p(ts), _p(w5), _p(ls), _p(gimg))
    assert rc == 0, rc
    return ls, gimg


def downsample(views, S, img, tile_w=16, tile_h=16, want_labels=True):
    """Fills levels >= 1 of every view from level 0 (img is modified in a copy)."""
    lib = _load()
    _, P, _ = layout(views, tile_w, tile_h)
    _, ci = Config(tile_w=tile_w, tile_h=tile_h).arrays(S)
    vi = _views(views)[1]
    out = _d(img).copy()
    lab = np.zeros(P, np.int32) if want_labels else None
    lib.or_downsample(_p(ci), ctypes.c_int(len(views)), _p(vi), _p(out), _p(lab))
    return out, lab


def sort_stage(views, n, m2hi, m2lo, radius, depth, tile_w=16, tile_h=16, cap=None):
    """Reference duplicate + sort + ranges on given single-precision projections."""
    lib = _load()
    _, _, tiles = layout(views, tile_w, tile_h)
    _, ci = Config(tile_w=tile_w, tile_h=tile_h).arrays(0)
    vi = _views(views)[1]
    m2hi = np.ascontiguousarray(m2hi, np.float32)
    m2lo = np.ascontiguousarray(m2lo, np.float32)
    radius = np.ascontiguousarray(radius, np.int32)
    depth = np.ascontiguousarray(depth, np.float32)
    if cap is None:
        cap = int(((2 * radius.astype(np.int64) // min(tile_w, tile_h) + 2) ** 2 * (radius > 0)).sum()) + 1
    keys = np.zeros(cap, np.uint64)
    vals = np.zeros(cap, np.uint32)
    ranges = np.zeros(2 * tiles, np.uint32)
    D = lib.or_sort_stage(_p(ci), ctypes.c_int(len(views)), _p(vi), ctypes.c_int64(n), _p(m2hi), _p(m2lo),
                          _p(radius), _p(depth), ctypes.c_int64(cap), _p(keys), _p(vals), _p(ranges))
    if D < 0:
        raise ValueError("capacity too small")
    return keys[:D], vals[:D], ranges.reshape(tiles, 2)


def distill(views, C, teacher, student, mse_w=0.1, tile_w=16, tile_h=16):
    """Distillation loss of student logits onto teacher logits ([P*C] planar per item)
    and its gradient with respect to the student."""
    lib = _load()
    _, P, _ = layout(views, tile_w, tile_h)
    _, ci = Config(tile_w=tile_w, tile_h=tile_h).arrays(0)
    vi = _views(views)[1]
    grad = np.zeros(P * C)
    loss = lib.or_distill(_p(ci), len(views), _p(vi), C, _p(_d(teacher)), _p(_d(student)), float(mse_w), _p(grad))
    return float(loss), grad


def head_forward(E, W1, b1, W2, b2):
    lib = _load()
    E = _d(E)
    P, D = E.shape
    Hd, C = W1.shape[0], W2.shape[0]
    out = np.zeros((P, C))
    lib.or_head_forward(ctypes.c_int64(P), ctypes.c_int(D), ctypes.c_int(Hd), ctypes.c_int(C), _p(E),
                        _p(_d(W1)), _p(_d(b1)), _p(_d(W2)), _p(_d(b2)), _p(out))
    return out


def head_backward(E, W1, b1, W2, dlogits):
    lib = _load()
    E = _d(E)
    P, D = E.shape
    Hd, C = W1.shape[0], W2.shape[0]
    dE = np.zeros((P, D))
    dW1 = np.zeros((Hd, D))
    db1 = np.zeros(Hd)
    dW2 = np.zeros((C, Hd))
    db2 = np.zeros(C)
    lib.or_head_backward(ctypes.c_int64(P), ctypes.c_int(D), ctypes.c_int(Hd), ctypes.c_int(C), _p(E),
                         _p(_d(W1)), _p(_d(b1)), _p(_d(W2)), _p(_d(dlogits)), _p(dE), _p(dW1), _p(db1),
                         _p(dW2), _p(db2))
    return dict(E=dE, W1=dW1, b1=db1, W2=dW2, b2=db2)
