"""Pins of the FP64 spherical-harmonics feature oracle: the basis against scipy's complex
harmonics and their orthonormality, its gradient, and the whole render with view-dependent
features against central differences (coefficients, means through the view direction,
and the pose through the camera centre)."""
import math

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import sh
from paper_2412_01217_amd import scenes


def _unit(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_basis_matches_scipy_real_harmonics_up_to_sign():
    rng = np.random.default_rng(40)
    d = _unit(rng, 200)
    polar = np.arccos(np.clip(d[:, 2], -1, 1))
    azim = np.arctan2(d[:, 1], d[:, 0])
    Y = sh.basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = special.sph_harm_y(l, abs(m), polar, azim)
            ref = c.real if m == 0 else math.sqrt(2) * (-1) ** m * (c.real if m > 0 else c.imag)
            ours = Y[:, l * l + l + m]
            s = np.sign(np.dot(ours, ref))                # the sign convention is free
            np.testing.assert_allclose(ours, s * ref, rtol=0, atol=1e-12, err_msg=f"l={l} m={m}")


def test_basis_is_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(polar) x uniform azimuth integrates these degree <= 6 products exactly
    x, w = np.polynomial.legendre.leggauss(8)
    az = np.arange(16) * 2 * np.pi / 16
    ct, ph = np.meshgrid(x, az, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).reshape(-1)
    Y = sh.basis(d, 3)
    np.testing.assert_allclose(Y.T @ (Y * wt[:, None]), np.eye(16), atol=1e-13)


def test_basis_gradient_matches_differences():
    rng = np.random.default_rng(41)
    d = rng.normal(size=(20, 3))
    G = sh.basis_grad(d, 3)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        fd = (sh.basis(d + e, 3) - sh.basis(d - e, 3)) / (2 * h)
        np.testing.assert_allclose(G[:, :, a], fd, atol=1e-8)


def test_degree_zero_is_the_plain_feature_and_features_are_linear():
    rng = np.random.default_rng(42)
    views = [scenes.identity_view(40, 30), scenes.View(np.eye(3), np.array([0.3, -0.1, 0.2]), 30, 30, 20, 15, 40, 30, 1)]
    mean = rng.normal(size=(7, 3)) + [0, 0, 3]
    dc = rng.normal(size=(7, 4))
    f = sh.features(views, mean, dc, None, 0)
    np.testing.assert_array_equal(f, np.stack([dc, dc]))
    r1, r2 = rng.normal(size=(7, 15, 4)), rng.normal(size=(7, 15, 4))
    lin = sh.features(views, mean, dc, r1 + 2 * r2, 3) - dc
    np.testing.assert_allclose(lin, (sh.features(views, mean, dc, r1, 3) - dc) + 2 * (sh.features(views, mean, dc, r2, 3) - dc),
                               atol=1e-13)


def _rodrigues(phi):
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th == 0:
        return np.eye(3)
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


@pytest.mark.parametrize("deg_rgb,deg_sem", [(3, 1), (2, 0)])
def test_render_with_view_dependent_features_matches_central_differences(deg_rgb, deg_sem):
    from oracle.mapping import exp_se3
    rng = np.random.default_rng(43 + deg_rgb)
    n, S = 8, 3
    mean = np.stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.3, 0.3, n), rng.uniform(1.5, 2.5, n)], 1)
    sc = scenes.Scene(mean, rng.normal(-2.3, 0.3, (n, 3)), rng.normal(size=(n, 4)), rng.normal(size=n) - 0.5,
                      rng.uniform(size=(n, 3)), rng.normal(size=(n, S)), None, S)
    views = [scenes.View(np.eye(3), np.zeros(3), 30.0, 30.0, 20.0, 16.0, 40, 32, 1),
             scenes.View(_rodrigues(np.array([0.04, -0.06, 0.03])), np.array([0.1, -0.05, 0.08]), 30.0, 30.0, 20.0, 16.0,
                         40, 32, 1)]
    cfg = oracle.Config().exact()
    rest_rgb = rng.normal(size=(n, sh.n_coeffs(deg_rgb) - 1, 3)) * 0.3
    rest_sem = rng.normal(size=(n, sh.n_coeffs(deg_sem) - 1, S)) * 0.3

    def run(mean_, rr, rs, vws):
        s = sc.copy()
        s.mean = mean_
        fr = sh.features(vws, mean_, sc.rgb, rr, deg_rgb)
        fs = sh.features(vws, mean_, sc.sem, rs, deg_sem)
        return sh.render(cfg, s, vws, fr, fs), fr, fs

    out, fr, fs = run(mean, rest_rgb, rest_sem, views)
    gimg = rng.normal(size=out["img"].shape)
    L = lambda *a: float(np.dot(gimg, run(*a)[0]["img"]))  # noqa: E731
    s0 = sc.copy()
    g = sh.backward(cfg, s0, views, fr, fs, gimg)
    _, grr, gm_r, gp_r = sh.features_backward(views, mean, rest_rgb, deg_rgb, g["rgb"])
    _, grs, gm_s, gp_s = sh.features_backward(views, mean, rest_sem, deg_sem, g["sem"])
    gmean = g["mean"] + gm_r + gm_s
    gpose = g["pose"] + gp_r + gp_s
    h = 1e-6
    fd_round = 50 * np.finfo(float).eps * abs(L(mean, rest_rgb, rest_sem, views)) / h

    def check(an, fd, what):
        scale = max(abs(fd), 1e-9)
        assert abs(an - fd) <= 1e-6 * scale + fd_round + 1e-10, (what, an, fd)

    for idx in list(np.ndindex(rest_rgb.shape))[::5]:
        e = np.zeros_like(rest_rgb); e[idx] = h
        check(grr[idx], (L(mean, rest_rgb + e, rest_sem, views) - L(mean, rest_rgb - e, rest_sem, views)) / (2 * h),
              ("rest_rgb", idx))
    if deg_sem > 0:
        for idx in list(np.ndindex(rest_sem.shape))[::3]:
            e = np.zeros_like(rest_sem); e[idx] = h
            check(grs[idx], (L(mean, rest_rgb, rest_sem + e, views) - L(mean, rest_rgb, rest_sem - e, views)) / (2 * h),
                  ("rest_sem", idx))
    for idx in np.ndindex(mean.shape):
        e = np.zeros_like(mean); e[idx] = h
        check(gmean[idx], (L(mean + e, rest_rgb, rest_sem, views) - L(mean - e, rest_rgb, rest_sem, views)) / (2 * h),
              ("mean", idx))
    for k in range(2):
        for j in range(6):
            xi = np.zeros(6); xi[j] = h
            vp, vm = list(views), list(views)
            for vv, sgn in ((vp, 1), (vm, -1)):
                Rd, td = exp_se3(sgn * xi)
                v = views[k]
                vv[k] = scenes.View(Rd @ v.R, Rd @ v.t + td, v.fx, v.fy, v.cx, v.cy, v.W, v.H, v.levels)
            check(gpose[k, j], (L(mean, rest_rgb, rest_sem, vp) - L(mean, rest_rgb, rest_sem, vm)) / (2 * h),
                  ("pose", k, j))
