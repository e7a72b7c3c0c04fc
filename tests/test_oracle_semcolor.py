"""Pins of the oracle's semantic colour loss (Sec. III-D eq. 12).

When the semantic feature is a colour (3 composited semantic channels), its loss has the form
of the RGB loss: (1 - lambda_s) mean |S - S_gt| over the 3HW values + lambda_s (1 - mean SSIM
of the 3 channels), the SSIM term read as 1 - SSIM as for eq. 10. These pins fix it by hand
values, against scipy's Gaussian filter (an implementation of SSIM independent of the
oracle's loops), by its constant-image closed form, by its independence from the RGB term
and by central differences of the whole loss.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import _ssim_scipy, view

S = 3   # semantic colour channels


def _img(W, H, sem, rng, rgb=None):
    """Image-layout buffer [7][H][W]: RGB (noise unless given), depth noise, semantic colour."""
    img = np.zeros((4 + S, H, W))
    img[:3] = rng.uniform(size=(3, H, W)) if rgb is None else rgb
    img[3] = rng.uniform(0.5, 2.0, size=(H, W))
    img[4:] = sem
    return img.reshape(-1)


def _loss(v, img, t_rgb, t_depth, t_sem, **kw):
    return oracle.loss([v], S, img, t_rgb, t_depth, None, t_sem=t_sem, **kw)


def test_semantic_colour_l1_hand_values_and_gradient():
    W, H = 4, 2
    v = view(W, H, 4.0)
    rng = np.random.default_rng(40)
    sem = np.zeros((3, H, W))
    sem[0] = 0.5
    sem[1] = [[0.0, 0.1, 0.2, 0.3], [0.4, 0.5, 0.6, 0.7]]
    sem[2] = 1.0
    t_sem = np.zeros((3, H, W))
    t_sem[0] = 1.0
    t_sem[1] = 0.25
    t_sem[2] = 1.0                                  # equal: sign 0, no gradient
    img = _img(W, H, sem, rng)
    ls, g = _loss(v, img, np.zeros(3 * 8), np.zeros(8), t_sem.reshape(-1), w=(1, 1, 2.0))
    # channel 0: 8 * 0.5; channel 1: |x - 0.25| summed = 0.25+0.15+0.05+0.05+0.15+0.25+0.35+0.45
    # = 1.7; channel 2: 0; over 3 * 8 values
    assert ls[0, 2] == pytest.approx((4.0 + 1.7) / 24, rel=1e-14)
    G = g.reshape(4 + S, H, W)
    np.testing.assert_allclose(G[4], -2.0 / 24)
    np.testing.assert_allclose(G[5], 2.0 / 24 * np.sign(sem[1] - 0.25))
    assert np.all(G[6] == 0)


def test_semantic_colour_ssim_matches_scipy():
    rng = np.random.default_rng(41)
    W, H = 23, 17
    v = view(W, H, 4.0)
    x, y = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    y[2] = 0.5 * x[2] + 0.3                         # a correlated channel
    for lam in (0.2, 1.0):
        ls, _ = _loss(v, _img(W, H, x, rng), rng.uniform(size=3 * W * H), np.ones(W * H), y.reshape(-1),
                      sem_ssim_lambda=lam)
        ssim = np.mean([_ssim_scipy(x[c], y[c]) for c in range(3)])
        assert ls[0, 2] == pytest.approx((1 - lam) * np.abs(x - y).mean() + lam * (1 - ssim), rel=1e-12)


def test_semantic_colour_ssim_constant_images():
    # constant semantic planes a and b on an image larger than the window: at the centre the
    # map is (2ab + C1) / (a^2 + b^2 + C1); identical images give loss 0 and zero gradient
    W, H = 14, 13
    v = view(W, H, 4.0)
    rng = np.random.default_rng(42)
    a, b = 0.7, 0.2
    C1 = 0.01 ** 2
    ls, _ = _loss(v, _img(W, H, np.full((3, H, W), a), rng), np.zeros(3 * W * H), np.ones(W * H),
                  np.full(3 * W * H, b), sem_ssim_lambda=1.0)
    centre = (2 * a * b + C1) / (a * a + b * b + C1)
    assert 0 < ls[0, 2] and 1 - ls[0, 2] < centre      # the border lowers the mean below the centre
    x = rng.uniform(size=(3, H, W))
    ls, g = _loss(v, _img(W, H, x, rng), np.zeros(3 * W * H), np.ones(W * H), x.reshape(-1),
                  w=(0, 0, 1), sem_ssim_lambda=1.0)
    assert abs(ls[0, 2]) < 1e-14
    assert np.abs(g.reshape(4 + S, H, W)[4:]).max() < 1e-13


def test_semantic_colour_term_is_the_rgb_term_on_other_channels():
    # eq. 12 has eq. 10's form: the semantic term of (sem, t_sem) equals the RGB term of the
    # same pair placed in the RGB planes, values and gradients, and the two terms do not mix
    rng = np.random.default_rng(43)
    W, H = 17, 12
    v = view(W, H, 4.0)
    x, y = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    lam = 0.3
    noise = rng.uniform(size=(3, H, W))
    ls_s, g_s = _loss(v, _img(W, H, x, rng, rgb=noise), noise.reshape(-1), np.ones(W * H), y.reshape(-1),
                      w=(1, 0, 1), ssim_lambda=0.6, sem_ssim_lambda=lam)
    ls_r, g_r = _loss(v, _img(W, H, y, rng, rgb=x), y.reshape(-1), np.ones(W * H), y.reshape(-1),
                      w=(1, 0, 1), ssim_lambda=lam, sem_ssim_lambda=0.6)
    assert ls_s[0, 2] == pytest.approx(ls_r[0, 0], rel=1e-13)
    assert abs(ls_s[0, 0]) < 1e-14 and abs(ls_r[0, 2]) < 1e-14   # identical pairs: zero
    Gs, Gr = g_s.reshape(4 + S, H, W), g_r.reshape(4 + S, H, W)
    np.testing.assert_allclose(Gs[4:], Gr[:3], rtol=1e-12, atol=1e-16)
    assert np.abs(Gs[:3]).max() < 1e-13 and np.abs(Gr[4:]).max() < 1e-13


def test_semantic_colour_loss_gradient_finite_difference():
    rng = np.random.default_rng(44)
    W, H = 13, 11
    HW = W * H
    v = view(W, H, 4.0)
    img = rng.uniform(size=(4 + S) * HW)
    t_rgb, t_depth, t_sem = rng.uniform(size=3 * HW), rng.uniform(0, 2, HW), rng.uniform(size=3 * HW)
    w, lam_r, lam_s = (0.7, 1.3, 0.9), 0.2, 0.35
    kw = dict(ssim_lambda=lam_r, sem_ssim_lambda=lam_s)
    _, g = _loss(v, img, t_rgb, t_depth, t_sem, w=w, **kw)
    L = lambda x: float(np.dot(w, _loss(v, x, t_rgb, t_depth, t_sem, **kw)[0][0]))  # noqa: E731
    h = 1e-6
    picks = list(rng.choice(np.arange(4 * HW, 7 * HW), 40, replace=False)) + [4 * HW, 5 * HW - 1, 7 * HW - 1]
    for j in picks + list(rng.choice(4 * HW, 10, replace=False)):
        e = np.zeros_like(img)
        e[j] = h
        fd = (L(img + e) - L(img - e)) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-6, abs=1e-9)


def test_semantic_colour_needs_three_channels():
    v = view(4, 2, 4.0)
    with pytest.raises(ValueError):
        oracle.loss([v], 4, np.zeros(8 * 8), np.zeros(24), np.zeros(8), None, t_sem=np.zeros(24))
