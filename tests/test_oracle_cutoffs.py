"""Pins of the oracle's cut-off rules with hand-computed values (paper Sec. III-C,
eq. 7-9, with the cut-offs read as in the 3DGS rasterizer the paper builds on).

The compositing of eq. 7-9 states no cut-offs; the build adds three (alpha below
alpha_min is skipped, alpha is clamped to alpha_max, a pixel stops before the
Gaussian that would take T below t_min), and the projection clamps x/z, y/z to the
guard band inside the Jacobian. Each case below sets its numbers so that the expected
image is exact in binary floating point, and so that the plausible slips -- "stop
after" for "stop before", <= for <, a skip that stops the pixel, no clamp, the wrong
guard limit -- each change the result.

Every Gaussian of the compositing cases sits on the optical axis with the principal
point at a pixel centre, so its offset there is exactly zero, the footprint exponent
is exactly 0 and alpha is exactly the opacity sigmoid(a); a = 0 gives exactly 1/2.
"""
import math

import numpy as np

import oracle
from paper_2412_01217_amd import scenes

W, H = 64, 48
CU, CV = 32, 24                  # the pixel whose centre (32.5, 24.5) is the principal point


def _scene(z, a, rgb, log_scale=-3.0):
    n = len(z)
    mean = np.zeros((n, 3))
    mean[:, 2] = z
    sem = np.zeros((n, 0))
    return scenes.Scene(mean, np.full((n, 3), float(log_scale)), np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                        np.asarray(a, np.float64), np.asarray(rgb, np.float64), sem, None, 0)


def _view():
    return scenes.View(np.eye(3), np.zeros(3), 50.0, 50.0, CU + 0.5, CV + 0.5, W, H, 1)


def _centre(out):
    """(rgb + depth at the centre pixel, T, n_contrib, blended count, flag)."""
    p = CV * W + CU
    img = out["img"].reshape(4, H, W)[:, CV, CU]
    return img, out["T"][p], out["n_contrib"][p], out["n_blend"][p], out["flag"][p]


RGB3 = [[0.25, 0.5, 0.75], [1.0, 0.125, 0.5], [0.5, 0.25, 1.0]]


def test_alpha_min_skips_exactly_below_threshold():
    # alpha_min = 1/2: the Gaussians with alpha = 1/2 are kept (alpha < alpha_min skips),
    # the middle one, alpha = sigmoid(-1) < 1/2, is skipped without stopping the pixel
    sc = _scene([2.0, 3.0, 4.0], [0.0, -1.0, 0.0], RGB3)
    cfg = oracle.Config(alpha_min=0.5, t_min=0.0)
    img, T, nc, nb, _ = _centre(oracle.render(cfg, sc, [_view()]))
    expect_rgb = [0.25 * 0.5 + 0.5 * 0.25, 0.5 * 0.5 + 0.25 * 0.25, 0.75 * 0.5 + 1.0 * 0.25]
    assert list(img[:3]) == expect_rgb
    assert img[3] == 2.0 * 0.5 + 4.0 * 0.25            # depth, eq. 8
    assert T == 0.25
    assert nc == 3                                      # 1 + position of the last blend
    assert nb == 2                                      # the skipped one is not blended


def test_default_alpha_min_skips_a_faint_gaussian():
    # default alpha_min = 1/255: opacity 0.003 is skipped, 0.005 is blended
    logit = lambda o: math.log(o / (1 - o))  # noqa: E731
    sc = _scene([2.0, 3.0, 4.0], [0.0, logit(0.003), logit(0.005)], RGB3)
    img, T, nc, nb, flag = _centre(oracle.render(oracle.Config(), sc, [_view()]))
    o3 = 1 / (1 + math.exp(-logit(0.005)))
    np.testing.assert_allclose(img[:3], 0.5 * np.array(RGB3[0]) + o3 * 0.5 * np.array(RGB3[2]), rtol=1e-15)
    np.testing.assert_allclose(T, 0.5 * (1 - o3), rtol=1e-15)
    assert (nc, nb, flag) == (3, 2, 0)


def test_stop_before_the_gaussian_that_would_take_t_below_t_min():
    # alpha = 1/2 four times: T goes 1 -> 1/2 -> 1/4 -> 1/8 -> 1/16. With t_min = 1/8 the
    # third Gaussian leaves T = 1/8 exactly (not below: blended) and the fourth would take
    # it to 1/16 < 1/8, so the pixel stops before the fourth.
    rgb = RGB3 + [[1.0, 1.0, 1.0]]
    sc = _scene([2.0, 3.0, 4.0, 5.0], [0.0, 0.0, 0.0, 0.0], rgb)
    cfg = oracle.Config(t_min=0.125)
    img, T, nc, nb, _ = _centre(oracle.render(cfg, sc, [_view()]))
    w = [0.5, 0.25, 0.125]
    expect_rgb = [sum(w[i] * rgb[i][c] for i in range(3)) for c in range(3)]
    assert list(img[:3]) == expect_rgb
    assert img[3] == 2.0 * 0.5 + 3.0 * 0.25 + 4.0 * 0.125
    assert T == 0.125
    assert (nc, nb) == (3, 3)
    # t_min = 0 blends all four
    img0, T0, nc0, _, _ = _centre(oracle.render(oracle.Config(t_min=0.0), sc, [_view()]))
    assert (T0, nc0) == (0.0625, 4)
    assert img0[0] == expect_rgb[0] + 0.0625 * 1.0


def test_alpha_max_clamp_value_and_zero_opacity_gradient():
    # opacity sigmoid(8) > 0.99 is clamped to alpha_max = 0.99; behind it alpha = 1/2
    sc = _scene([2.0, 3.0], [8.0, 0.0], RGB3[:2])
    cfg = oracle.Config()
    v = _view()
    img, T, nc, _, _ = _centre(oracle.render(cfg, sc, [v]))
    a1 = 0.99
    np.testing.assert_allclose(img[:3], a1 * np.array(RGB3[0]) + 0.5 * (1 - a1) * np.array(RGB3[1]), rtol=1e-15)
    np.testing.assert_allclose(T, (1 - a1) * 0.5, rtol=1e-15)
    assert nc == 2
    # d(centre red)/d(logit) is zero through the clamp for the front Gaussian (the derivative
    # at a kink is read as 0), and that of the Gaussian behind it is d(0.5 (1 - 0.99) r)/da
    gimg = np.zeros(4 * W * H)
    gimg[0 * W * H + CV * W + CU] = 1.0
    g = oracle.backward(cfg, sc, [v], gimg)
    assert g["opacity"][0] == 0.0
    o2 = 0.5
    np.testing.assert_allclose(g["opacity"][1], (1 - a1) * RGB3[1][0] * o2 * (1 - o2), rtol=1e-12)


def test_near_threshold_decisions_are_flagged():
    # alpha within the oracle's margin of alpha_min, and T within it of t_min
    eps = 1e-7
    a = math.log((0.5 + eps) / (0.5 - eps))           # sigmoid(a) = 1/2 + eps
    sc = _scene([2.0, 3.0], [a, 0.0], RGB3[:2])
    _, _, _, _, flag = _centre(oracle.render(oracle.Config(alpha_min=0.5, t_min=0.0), sc, [_view()]))
    assert flag & 1
    sc2 = _scene([2.0, 3.0, 4.0], [0.0, 0.0, 0.0], RGB3)
    _, _, _, _, flag2 = _centre(oracle.render(oracle.Config(t_min=0.125 * (1 + 1e-6)), sc2, [_view()]))
    assert flag2 & 4
    _, _, _, _, flag3 = _centre(oracle.render(oracle.Config(t_min=0.1), sc2, [_view()]))
    assert flag3 == 0


def _cov_closed_form(s, z, fx, fy, ux, uy, eps):
    # isotropic Sigma = s^2 I: J Sigma J^T + eps I with J at the (clamped) ux = x/z, uy = y/z
    a = s * s * (fx / z) ** 2 * (1 + ux * ux) + eps
    b = s * s * fx * fy / z ** 2 * ux * uy
    c = s * s * (fy / z) ** 2 * (1 + uy * uy) + eps
    return a, b, c


def test_guard_band_clamps_the_jacobian_only():
    # x/z and y/z are clamped to +-guard (W/2)/fx and +-guard (H/2)/fy inside J; the mean
    # itself projects unclamped. fx != fy and W != H so that a limit taken from the other
    # axis fails; ratios 1.1 (clamped) and 0.9, 0.95 (not) separate the limit from a
    # doubled or guard-free one.
    Wv, Hv, fx, fy = 64, 48, 50.0, 40.0
    limx, limy = 1.3 * (Wv / 2) / fx, 1.3 * (Hv / 2) / fy
    z = 2.0
    ratios = [(1.1 * limx, 0.2), (0.9 * limx, -1.2 * limy), (0.95 * limx, 0.95 * limy), (-1.5 * limx, 1.05 * limy)]
    mean = np.array([[rx * z, ry * z, z] for rx, ry in ratios])
    s = 0.05
    n = len(ratios)
    sc = scenes.Scene(mean, np.full((n, 3), math.log(s)), np.tile([0.9, 0.1, -0.3, 0.2], (n, 1)), np.zeros(n),
                      np.ones((n, 3)), np.zeros((n, 0)), None, 0)
    v = scenes.View(np.eye(3), np.zeros(3), fx, fy, Wv / 2, Hv / 2, Wv, Hv, 1)
    cfg = oracle.Config(full_rect=True)
    pp = oracle.preprocess(cfg, sc, [v])
    assert np.all(pp["radius"] > 0)
    for k, (rx, ry) in enumerate(ratios):
        ux, uy = max(-limx, min(limx, rx)), max(-limy, min(limy, ry))
        a, b, c = _cov_closed_form(s, z, fx, fy, ux, uy, cfg.eps)
        det = a * c - b * b
        np.testing.assert_allclose(pp["conic"][k], [c / det, -b / det, a / det], rtol=1e-12)
        np.testing.assert_allclose(pp["m2"][k], [fx * rx + Wv / 2, fy * ry + Hv / 2], rtol=1e-14)
        if (ux, uy) != (rx, ry):      # the unclamped covariance is measurably different
            a2, b2, c2 = _cov_closed_form(s, z, fx, fy, rx, ry, cfg.eps)
            assert abs(a2 - a) + abs(b2 - b) + abs(c2 - c) > 1e-3 * (abs(a) + abs(c))


def test_box_pyramid_hand_values():
    # one 4 x 2 view with 2 levels (level 1 is 2 x 1), rgb + depth + 2 logits
    v = scenes.View(np.eye(3), np.zeros(3), 10.0, 10.0, 2.0, 1.0, 4, 2, 2)
    K = 6
    lv0 = np.array([
        [[1, 2, 3, 4], [5, 6, 7, 8]],          # R
        [[0, 0, 1, 1], [0, 0, 1, -1]],         # G
        [[-2, 2, 0.5, 0.5], [1, 1, 0, 0]],     # B
        [[1, 0, 2, 2], [0, 0, 4, 0]],          # depth: zeros are missing values
        [[1, 1, 0, 0], [1, 1, 0, 0]],          # logit 0
        [[0, 2, 0, 1], [2, 0, 1, 0]],          # logit 1
    ], np.float64)
    img = np.zeros(K * (8 + 2))
    img[:K * 8] = lv0.reshape(-1)
    out, lab = oracle.downsample([v], 2, img)
    lv1 = out[K * 8:].reshape(K, 1, 2)
    expect = [[3.5, 5.5], [0.0, 0.5], [0.5, 0.25], [1.0, 8.0 / 3.0], [1.0, 0.0], [1.0, 0.5]]
    for c in range(K):
        np.testing.assert_allclose(lv1[c, 0], expect[c], rtol=1e-15)
    # labels: argmax over the logits, ties to the lower class
    np.testing.assert_array_equal(lab[:8], [0, 1, 0, 1, 1, 0, 1, 0])
    np.testing.assert_array_equal(lab[8:], [0, 1])
