"""Test infrastructure: FP64 reference of view-dependent features by spherical harmonics
(paper Sec. III-B: colour and semantic features of each Gaussian represented with SH).

Per view v and Gaussian i the feature of channel c is

    f_vic = dc_ic + sum over 1 <= l <= degree, -l <= m <= l of Y_lm(d_vi) k_i,lm,c

with d_vi = (mu_i - c_v) / |mu_i - c_v| the unit direction from the camera centre
c_v = -R_v^T t_v to the Gaussian (world frame), and Y_lm the real spherical harmonics in
the sign convention of the 3DGS renderer the paper builds on. The constant band is the
plain feature itself, so degree 0 gives the view-independent features.

Only the tests import this module; nothing is shared with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

# normalisation constants of the real spherical harmonics (Condon-Shortley phase folded in)
_C1 = math.sqrt(3.0 / (4.0 * math.pi))
_C2 = (math.sqrt(15.0 / math.pi) / 2.0, -math.sqrt(15.0 / math.pi) / 2.0, math.sqrt(5.0 / math.pi) / 4.0,
       -math.sqrt(15.0 / math.pi) / 2.0, math.sqrt(15.0 / math.pi) / 4.0)
_C3 = (-math.sqrt(35.0 / (2.0 * math.pi)) / 4.0, math.sqrt(105.0 / math.pi) / 2.0,
       -math.sqrt(21.0 / (2.0 * math.pi)) / 4.0, math.sqrt(7.0 / math.pi) / 4.0,
       -math.sqrt(21.0 / (2.0 * math.pi)) / 4.0, math.sqrt(105.0 / math.pi) / 4.0,
       -math.sqrt(35.0 / (2.0 * math.pi)) / 4.0)
Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def n_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def basis(d, degree: int):
    """Y_j(d), j = l^2 + l + m, for unit directions d [..., 3] -> [..., (degree+1)^2]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full(x.shape, Y00)]
    if degree >= 1:
        out += [-_C1 * y, _C1 * z, -_C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [_C2[0] * x * y, _C2[1] * y * z, _C2[2] * (2 * zz - xx - yy), _C2[3] * x * z, _C2[4] * (xx - yy)]
    if degree >= 3:
        xx, yy, zz = x * x, y * y, z * z
        out += [_C3[0] * y * (3 * xx - yy), _C3[1] * x * y * z, _C3[2] * y * (4 * zz - xx - yy),
                _C3[3] * z * (2 * zz - 3 * xx - 3 * yy), _C3[4] * x * (4 * zz - xx - yy), _C3[5] * z * (xx - yy),
                _C3[6] * x * (xx - 3 * yy)]
    return np.stack(out, -1)


def basis_grad(d, degree: int):
    """dY_j/dd (the polynomials' gradient in the ambient 3D coordinates) -> [..., K, 3]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    g = [(zero, zero, zero)]
    if degree >= 1:
        c = np.full(x.shape, _C1)
        g += [(zero, -c, zero), (zero, zero, c), (-c, zero, zero)]
    if degree >= 2:
        g += [(_C2[0] * y, _C2[0] * x, zero), (zero, _C2[1] * z, _C2[1] * y),
              (-2 * _C2[2] * x, -2 * _C2[2] * y, 4 * _C2[2] * z), (_C2[3] * z, zero, _C2[3] * x),
              (2 * _C2[4] * x, -2 * _C2[4] * y, zero)]
    if degree >= 3:
        xx, yy, zz = x * x, y * y, z * z
        g += [(_C3[0] * 6 * x * y, _C3[0] * (3 * xx - 3 * yy), zero),
              (_C3[1] * y * z, _C3[1] * x * z, _C3[1] * x * y),
              (_C3[2] * (-2 * x * y), _C3[2] * (4 * zz - xx - 3 * yy), _C3[2] * 8 * y * z),
              (_C3[3] * (-6 * x * z), _C3[3] * (-6 * y * z), _C3[3] * (6 * zz - 3 * xx - 3 * yy)),
              (_C3[4] * (4 * zz - 3 * xx - yy), _C3[4] * (-2 * x * y), _C3[4] * 8 * x * z),
              (_C3[5] * 2 * x * z, _C3[5] * (-2 * y * z), _C3[5] * (xx - yy)),
              (_C3[6] * (3 * xx - 3 * yy), _C3[6] * (-6 * x * y), zero)]
    return np.stack([np.stack(t, -1) for t in g], -2)


def camera_centre(v):
    R = np.asarray(v.R, np.float64).reshape(3, 3)
    return -R.T @ np.asarray(v.t, np.float64)


def features(views, mean, dc, rest, degree):
    """[V][N][ch] features; rest [N][(degree+1)^2 - 1][ch] (ignored for degree 0)."""
    mean = np.asarray(mean, np.float64)
    dc = np.asarray(dc, np.float64)
    out = []
    for v in views:
        u = mean - camera_centre(v)
        d = u / np.linalg.norm(u, axis=1, keepdims=True)
        f = dc.copy()
        if degree > 0:
            Y = basis(d, degree)[:, 1:]                                  # [N][K-1]
            f = f + np.einsum("nk,nkc->nc", Y, np.asarray(rest, np.float64))
        out.append(f)
    return np.stack(out)


def features_backward(views, mean, rest, degree, gfeat):
    """Gradients of sum gfeat . features: (d dc [N][ch], d rest, d mean [N][3], d pose [V][6]).
    The pose tangent is the left perturbation T_cw <- Exp(xi) T_cw; the camera centre moves by
    -R^T rho and not with phi."""
    mean = np.asarray(mean, np.float64)
    gfeat = np.asarray(gfeat, np.float64)
    gdc = gfeat.sum(0)
    grest = np.zeros_like(np.asarray(rest, np.float64)) if degree > 0 else None
    gmean = np.zeros_like(mean)
    gpose = np.zeros((len(views), 6))
    if degree == 0:
        return gdc, grest, gmean, gpose
    rest = np.asarray(rest, np.float64)
    for k, v in enumerate(views):
        u = mean - camera_centre(v)
        r = np.linalg.norm(u, axis=1, keepdims=True)
        d = u / r
        Y = basis(d, degree)[:, 1:]
        grest += Y[:, :, None] * gfeat[k][:, None, :]
        dY = basis_grad(d, degree)[:, 1:]                              # [N][K-1][3]
        gd = np.einsum("nc,nkc,nkj->nj", gfeat[k], rest, dY)           # d L / d d
        gu = (gd - d * np.sum(d * gd, 1, keepdims=True)) / r            # through the normalisation
        gmean += gu
        R = np.asarray(v.R, np.float64).reshape(3, 3)
        gpose[k, :3] = R @ gu.sum(0)                                    # c = -R^T t, dc/drho = -R^T
    return gdc, grest, gmean, gpose


def render(cfg, scene, views, rgb_v, sem_v):
    """Oracle render with per-view features: every view rendered with its own rgb [N][3] and
    sem [N][S]; the outputs concatenated in the item layout (items are view-major)."""
    imgs, Ts, ncs, flags = [], [], [], []
    for k, v in enumerate(views):
        s = scene.copy()
        s.rgb = np.asarray(rgb_v[k], np.float64)
        s.sem = np.asarray(sem_v[k], np.float64)
        out = oracle.render(cfg, s, [v])
        imgs.append(out["img"]); Ts.append(out["T"]); ncs.append(out["n_contrib"]); flags.append(out["flag"])
    return dict(img=np.concatenate(imgs), T=np.concatenate(Ts), n_contrib=np.concatenate(ncs),
                flag=np.concatenate(flags), K=4 + np.asarray(sem_v).shape[2])


def backward(cfg, scene, views, rgb_v, sem_v, gimg):
    """Oracle backward with per-view features: per-view feature gradients [V][N][ch], the
    geometric gradients summed over views, and each view's pose gradient."""
    K = 4 + np.asarray(sem_v).shape[2]
    its = oracle.items(views)
    out = dict(rgb=[], sem=[], pose=np.zeros((len(views), 6)))
    acc = {}
    for k, v in enumerate(views):
        s = scene.copy()
        s.rgb = np.asarray(rgb_v[k], np.float64)
        s.sem = np.asarray(sem_v[k], np.float64)
        mine = [it for it in its if it["view"] == k]
        a = mine[0]["pix0"] * K
        b = (mine[-1]["pix0"] + mine[-1]["W"] * mine[-1]["H"]) * K
        g = oracle.backward(cfg, s, [v], np.asarray(gimg)[a:b])
        out["rgb"].append(g["rgb"])
        out["sem"].append(g["sem"])
        out["pose"][k] = g["pose"][0]
        for name in ("mean", "log_scale", "quat", "opacity"):
            acc[name] = acc.get(name, 0) + g[name]
    out.update(acc)
    out["rgb"] = np.stack(out["rgb"])
    out["sem"] = np.stack(out["sem"])
    return out
