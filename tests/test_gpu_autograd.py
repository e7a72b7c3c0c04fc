"""The autograd.Function's backward against FP64 central finite differences.

For L = sum(gimg * render(theta)), 64 parameters drawn from Gaussians visible in
the image (every parameter group) plus the six pose-tangent components are checked:
|g_gpu - g_fd| <= 1e-3 * max(|g_fd|, 0.01 rms(group)), with g_fd from the FP64
oracle at theta +- h, h = 1e-4. A draw whose +-h perturbation changes a discrete
decision of the oracle (which Gaussians a pixel blends, radius or tile rectangle)
is replaced by another draw.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_01217_amd import scenes
from tests.helpers import pixel_mask_to_channels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = 1e-4
TOL = 1e-3


def _rodrigues(phi):
    th = np.linalg.norm(phi)
    Kx = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-300:
        return np.eye(3) + Kx
    return np.eye(3) + math.sin(th) / th * Kx + (1 - math.cos(th)) / th ** 2 * Kx @ Kx


def _exp_se3(xi):
    rho, phi = xi[:3], xi[3:]
    th = np.linalg.norm(phi)
    R = _rodrigues(phi)
    Kx = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    V = np.eye(3) + 0.5 * Kx if th < 1e-12 else \
        np.eye(3) + (1 - math.cos(th)) / th ** 2 * Kx + (th - math.sin(th)) / th ** 3 * Kx @ Kx
    return R, V @ rho


def _double(sc):
    return scenes.Scene(*(np.asarray(getattr(sc, f), np.float64) for f in
                          ("mean", "log_scale", "quat", "opacity", "rgb", "sem")), None, sc.n_classes)


def test_autograd_backward_matches_fp64_finite_differences():
    from paper_2412_01217_amd import autograd, raster
    sc32, views = scenes.config_tiny()
    v = views[0]
    v = scenes.View(_rodrigues(np.array([0.03, -0.02, 0.04])).astype(np.float32),
                    np.array([0.02, -0.03, 0.05], np.float32), v.fx, v.fy, v.cx, v.cy, v.W, v.H, v.levels)
    views = [v]
    sc = _double(sc32)
    cfg_o = oracle.Config()
    base = oracle.render(cfg_o, sc, views)
    K = base["K"]
    rng = np.random.default_rng(5300)
    gimg = rng.normal(size=base["img"].shape)
    gimg[pixel_mask_to_channels(base["flag"] != 0, oracle.items(views), K)] = 0.0

    cfg = raster.config(sc32.n_classes)
    fr = raster.Frame(cfg, views)
    t = {k: torch.tensor(np.asarray(getattr(sc32, k)), device="cuda", requires_grad=True)
         for k in ("mean", "log_scale", "quat", "opacity", "rgb", "sem")}
    xi = torch.zeros(1, 6, device="cuda", requires_grad=True)
    color, _, _ = autograd.render(t, fr, cfg, pose_xi=xi)
    loss = (color * torch.from_numpy(gimg).float().cuda()).sum()
    loss.backward()
    grads = {k: t[k].grad.cpu().numpy().astype(np.float64) for k in t}
    grads["pose"] = xi.grad.cpu().numpy().astype(np.float64)

    pre = oracle.preprocess(cfg_o, sc, views)
    visible = np.flatnonzero(pre["radius"] > 0)

    def decisions(s, vv):
        r = oracle.render(cfg_o, s, vv)
        p = oracle.preprocess(cfg_o, s, vv)
        return r, (r["n_contrib"].copy(), r["n_blend"].copy(), p["radius"].copy(), p["rect"].copy())

    def fd_of(make):
        rp, dp = decisions(*make(+H))
        rm, dm = decisions(*make(-H))
        same = (all(np.array_equal(a, b) for a, b in zip(dp, dm)) and np.array_equal(dp[0], base["n_contrib"])
                and np.array_equal(dp[1], base["n_blend"]))
        return float(np.dot(gimg, rp["img"] - rm["img"])) / (2 * H), same

    shapes = {"mean": 3, "log_scale": 3, "quat": 4, "opacity": 1, "rgb": 3, "sem": sc.n_classes}
    names = list(shapes)
    checked, redrawn = 0, 0
    while checked < 64:
        name = names[checked % len(names)]
        i = int(rng.choice(visible))
        c = int(rng.integers(shapes[name]))
        idx = (i, c) if name != "opacity" else (i,)

        def make(d, name=name, idx=idx):
            s2 = sc.copy()
            getattr(s2, name)[idx] += d
            return s2, views

        fd, same = fd_of(make)
        if not same:
            redrawn += 1
            assert redrawn < 64, "too many draws cross a decision"
            continue
        g = grads[name][idx]
        scale = max(abs(fd), 0.01 * float(np.sqrt(np.mean(grads[name] ** 2))))
        assert abs(g - fd) <= TOL * scale, (name, idx, g, fd)
        checked += 1
    # pose tangent: left perturbation Exp(xi) T_cw
    for j in range(6):
        def make(d, j=j):
            e = np.zeros(6)
            e[j] = d
            Rx, tx = _exp_se3(e)
            vv = scenes.View(Rx @ np.asarray(v.R, np.float64), Rx @ np.asarray(v.t, np.float64) + tx,
                             v.fx, v.fy, v.cx, v.cy, v.W, v.H, v.levels)
            return sc, [vv]

        fd, same = fd_of(make)
        if not same:
            continue
        g = grads["pose"][0, j]
        scale = max(abs(fd), 0.01 * float(np.sqrt(np.mean(grads["pose"] ** 2))))
        assert abs(g - fd) <= TOL * scale, ("pose", j, g, fd)


def test_autograd_twice_gives_same_gradients():
    from paper_2412_01217_amd import autograd, raster
    sc, views = scenes.config_tiny()
    cfg = raster.config(sc.n_classes)
    fr = raster.Frame(cfg, views)
    gimg = torch.from_numpy(scenes.random_image(fr.n_pixels, 12, seed=5301)).cuda()
    out = []
    for _ in range(2):
        t = {k: torch.tensor(np.asarray(getattr(sc, k)), device="cuda", requires_grad=True)
             for k in ("mean", "log_scale", "quat", "opacity", "rgb", "sem")}
        color, _, _ = autograd.render(t, fr, cfg)
        (color * gimg).sum().backward()
        out.append({k: t[k].grad.clone() for k in t})
    # float atomics may add in another order from run to run
    for k in out[0]:
        torch.testing.assert_close(out[0][k], out[1][k], rtol=1e-4, atol=1e-7)
