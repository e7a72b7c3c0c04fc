"""ctypes mirror of include/gs.h and the loader of libgs.so.

Marshalling only: every computation happens in the HIP library. Importing this
module does not touch the GPU; `lib()` raises if libgs.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_uint16, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_WORKSPACE = -2
GS_ERR_CAPACITY = -3
GS_ERR_HIP = -4
GS_ERR_UNSUPPORTED = -5

GS_WS_BIN_SORT = 1
GS_WS_RENDER_BWD = 2
GS_WS_LOSS = 3
GS_WS_RENDER_STATE = 4

# Every symbol include/gs.h declares.
EXPORTS = (
    "gs_config_default", "gs_status_string", "gs_last_hip_error", "gs_version", "gs_make_items",
    "gs_workspace_size", "gs_preprocess", "gs_bin_sort", "gs_render_fwd", "gs_pyramid_loss",
    "gs_render_bwd", "gs_pyramid_downsample", "gs_graph_begin", "gs_graph_end", "gs_graph_launch",
    "gs_graph_destroy", "gs_adam_step", "gs_distill_loss", "gs_argmax_agreement", "gs_gaussians_adam",
    "gs_pose_adam", "gs_sh_features", "gs_sh_features_bwd", "gs_pose_perturb", "gs_pose_perturb_bwd",
    "gs_pyramid_loss_static",
)


class Config(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("z_near", c_float), ("eps_dilate", c_float),
                ("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float), ("guard", c_float),
                ("full_rect", c_int32), ("n_sem", c_int32), ("variant", c_int32), ("tile_order", c_int32),
                ("fwd_chunk", c_int32), ("ssim_lambda", c_float), ("isotropic", c_int32),
                ("view_features", c_int32), ("sem_ssim_lambda", c_float), ("seg_len", c_int32), ("sort_mode", c_int32)]


class View(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("item_first", c_int32), ("item_count", c_int32)]


class Item(ctypes.Structure):
    _fields_ = [("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float), ("W", c_int32), ("H", c_int32),
                ("view", c_int32), ("level", c_int32), ("tiles_x", c_int32), ("tiles_y", c_int32),
                ("tile_base", c_int32), ("pad", c_int32), ("pixel_base", c_int64)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p),
                ("opacity", c_void_p), ("rgb", c_void_p), ("sem", c_void_p), ("emb", c_void_p)]


class Projected(ctypes.Structure):
    _fields_ = [("rec", c_void_p), ("depth", c_void_p), ("radius", c_void_p)]


class Images(ctypes.Structure):
    _fields_ = [("color", c_void_p), ("T", c_void_p), ("n_contrib", c_void_p), ("logits", c_void_p),
                ("n_pixels", c_int64), ("state", c_void_p), ("state_bytes", ctypes.c_size_t)]


class Targets(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("label", c_void_p), ("sem_color", c_void_p)]


class ParamArrays(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p), ("opacity", c_void_p),
                ("rgb", c_void_p), ("sem", c_void_p)]


class SH(ctypes.Structure):
    _fields_ = [("rgb_degree", c_int32), ("sem_degree", c_int32), ("rgb_rest", c_void_p), ("sem_rest", c_void_p)]


class AdamConfig(ctypes.Structure):
    _fields_ = [(k, c_float) for k in ("lr_mean", "lr_log_scale", "lr_quat", "lr_opacity", "lr_rgb", "lr_sem",
                                       "lr_rho", "lr_phi", "beta1", "beta2", "eps")]


class Head(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("d_hidden", c_int32), ("n_classes", c_int32), ("pad", c_int32),
                ("W1", c_void_p), ("b1", c_void_p), ("W2", c_void_p), ("b2", c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p), ("opacity", c_void_p),
                ("rgb", c_void_p), ("sem", c_void_p), ("emb", c_void_p), ("pose", c_void_p),
                ("head_W1", c_void_p), ("head_b1", c_void_p), ("head_W2", c_void_p), ("head_b2", c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P = POINTER
        L.gs_config_default.argtypes = [P(Config)]
        L.gs_config_default.restype = None
        L.gs_status_string.argtypes = [c_int32]
        L.gs_status_string.restype = ctypes.c_char_p
        L.gs_last_hip_error.restype = c_int32
        L.gs_version.restype = c_int32
        L.gs_make_items.argtypes = [P(Config), c_int32, P(View), P(c_int32), P(c_int32), P(c_float), P(c_int32),
                                    P(Item), P(c_int64), P(c_int32)]
        L.gs_workspace_size.argtypes = [c_int32, P(Config), c_int32, c_int64, c_int32, c_int64, c_int64, P(c_size_t)]
        L.gs_preprocess.argtypes = [P(Config), P(Gaussians), c_void_p, c_int32, c_void_p, c_int32, P(Projected),
                                    c_void_p]
        L.gs_bin_sort.argtypes = [P(Config), P(Projected), c_void_p, c_int32, c_int64, c_int32, c_int64, c_void_p,
                                  c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.gs_render_fwd.argtypes = [P(Config), P(Gaussians), P(Projected), c_void_p, c_int32, c_int32, c_void_p,
                                    c_void_p, c_void_p, P(Images), c_void_p]
        L.gs_pyramid_loss.argtypes = [P(Config), c_void_p, c_int32, c_int64, c_int32, P(Images), P(Targets),
                                      c_void_p, P(c_float), c_void_p, P(Images), c_void_p, c_void_p, c_size_t, c_void_p]
        L.gs_render_bwd.argtypes = [P(Config), P(Gaussians), P(Projected), c_void_p, c_int32, c_void_p, c_int32,
                                    c_int32, c_void_p, c_void_p, c_void_p, P(Images), P(Images), P(Grads), c_void_p,
                                    c_size_t, c_void_p]
        L.gs_pyramid_downsample.argtypes = [c_void_p, c_int32, c_int64, c_int32, c_int32, c_void_p, c_void_p,
                                            c_void_p]
        L.gs_adam_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_float, c_float, c_float,
                                   c_int32, c_void_p, c_void_p]
        L.gs_distill_loss.argtypes = [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_void_p, c_float, c_void_p,
                                      c_void_p, c_void_p, c_size_t, c_void_p]
        L.gs_argmax_agreement.argtypes = [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
        L.gs_gaussians_adam.argtypes = [c_int64, c_int32, P(ParamArrays), P(Grads), P(ParamArrays), P(ParamArrays),
                                        P(AdamConfig), c_int32, c_void_p]
        L.gs_pose_adam.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, P(AdamConfig), c_int32, c_void_p]
        L.gs_sh_features.argtypes = [c_int32, P(Gaussians), P(SH), c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
        L.gs_sh_features_bwd.argtypes = [c_int32, P(Gaussians), P(SH), c_void_p, c_int32] + [c_void_p] * 9
        L.gs_pose_perturb.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
        L.gs_pyramid_loss_static.argtypes = [P(Config), c_void_p, c_int32, c_int64, c_int32, P(Images), P(Targets),
                                             c_void_p, P(c_float), c_void_p, P(Images), c_void_p, c_void_p]
        L.gs_pose_perturb_bwd.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
        for name in ("gs_adam_step", "gs_distill_loss", "gs_argmax_agreement", "gs_gaussians_adam", "gs_pose_adam",
                     "gs_sh_features", "gs_sh_features_bwd", "gs_pose_perturb", "gs_pose_perturb_bwd",
                     "gs_pyramid_loss_static"):
            getattr(L, name).restype = c_int32
        L.gs_graph_begin.argtypes = [c_void_p]
        L.gs_graph_end.argtypes = [c_void_p, P(c_void_p)]
        L.gs_graph_launch.argtypes = [c_void_p, c_void_p]
        L.gs_graph_destroy.argtypes = [c_void_p]
        for name in ("gs_make_items", "gs_workspace_size", "gs_preprocess", "gs_bin_sort", "gs_render_fwd",
                     "gs_pyramid_loss", "gs_render_bwd", "gs_pyramid_downsample", "gs_graph_begin", "gs_graph_end",
                     "gs_graph_launch", "gs_graph_destroy"):
            getattr(L, name).restype = c_int32
        _lib = L
    return _lib


class GSError(RuntimeError):
    pass


def check(status: int, what: str) -> None:
    if status != GS_OK:
        L = lib()
        msg = L.gs_status_string(status).decode()
        if status == GS_ERR_HIP:
            msg += f" (hipError {L.gs_last_hip_error()})"
        raise GSError(f"{what}: {msg} [{status}]")
