"""GPU parity of the semantic colour loss (Sec. III-D eq. 12) against the oracle.

The semantic feature is a 3-channel colour composited like the RGB colour (plain mode with
3 semantic channels); its loss is (1 - lambda_s) L1 + lambda_s (1 - SSIM) against a semantic
colour target. Checked on the loss alone (random images over a 3-level pyramid with ragged
SSIM tiles, and items smaller than the window) and end to end through the render, the loss
and the backward to every Gaussian parameter and the pose, at the paper's lambda_r =
lambda_s = 0.2.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_01217_amd import scenes
from tests.helpers import flagged, over_limit, pixel_term_magnitude, rel_check, targets_from_random
from tests.test_gpu_parity import BWD_TOL, FWD_TOL, SSIM_VIEWS, _check_render_fwd, _pipeline, _raster, small_room

pytestmark = pytest.mark.gpu


def _sem_targets(views, seed):
    t_rgb, t_depth, _ = targets_from_random(views, 3, seed=seed)
    rng = np.random.default_rng(seed + 1)
    t_sem = rng.uniform(0.0, 1.0, size=t_rgb.shape).astype(np.float32)
    return t_rgb, t_depth, t_sem


@pytest.mark.parametrize("lams", [(0.0, 0.2), (0.2, 0.2), (0.0, 1.0), (0.3, 0.0)])
@pytest.mark.parametrize("case", list(SSIM_VIEWS))
def test_semantic_colour_loss_parity(case, lams):
    lam_r, lam_s = lams
    raster = _raster()
    views = SSIM_VIEWS[case]()
    cfg = raster.config(3, ssim_lambda=lam_r, sem_ssim_lambda=lam_s)
    fr = raster.Frame(cfg, views)
    img = scenes.random_image(fr.n_pixels, 7, seed=5110)
    t_rgb, t_depth, t_sem = _sem_targets(views, 4010)
    w = (0.8, 1.1, 0.6)
    ls_ref, g_ref = oracle.loss(views, 3, img, t_rgb, t_depth, None, w=w, ssim_lambda=lam_r, t_sem=t_sem,
                                sem_ssim_lambda=lam_s)
    T = dict(rgb=torch.from_numpy(t_rgb).cuda(), depth=torch.from_numpy(t_depth).cuda(),
             sem_color=torch.from_numpy(t_sem).cuda())
    rendered = dict(color=torch.from_numpy(img).cuda())
    ls, grad = raster.loss(cfg, fr, 0, rendered, T, w=w)
    torch.cuda.synchronize()
    rel_check(ls.cpu().numpy(), ls_ref, FWD_TOL, name="loss")
    rel_check(grad["color"].cpu().numpy(), g_ref, BWD_TOL, name="dloss/dimg")
    # a second call: every call clears the slots it sums into
    ls2, _ = raster.loss(cfg, fr, 0, rendered, T, w=w)
    torch.cuda.synchronize()
    np.testing.assert_allclose(ls2.cpu().numpy(), ls.cpu().numpy(), rtol=1e-6)


@pytest.mark.parametrize("scene", ["tiny", "room"])
def test_semantic_colour_end_to_end(scene):
    """Render (3 semantic colour channels), eq. 10-13 with eq. 12's semantic term at
    lambda_r = lambda_s = 0.2, backward; against the oracle's render, loss and backward."""
    if scene == "tiny":
        sc, views = scenes.config_tiny()
    else:
        sc, views = small_room()
    sc = scenes.semantic_colour_scene(sc)
    cfg, fr, g, proj, srt, img = _pipeline(sc, views, 3)
    cfg.ssim_lambda = 0.2
    cfg.sem_ssim_lambda = 0.2
    raster = _raster()
    ocfg = oracle.Config()
    r = oracle.render(ocfg, sc, views)
    _check_render_fwd(sc, views, 3, True)     # the semantic colour image composited like RGB
    # targets at least 0.02 from the render in every channel, so that the L1 terms' signs are
    # the same for the single-precision render and the oracle's (R13: a sign at the kink is
    # a discrete choice); a tenth of the depths missing
    rng = np.random.default_rng(4020)
    t_rgb, t_depth, t_sem = [], [], []
    for it in oracle.items(views):
        HW = it["W"] * it["H"]
        im = r["img"][it["pix0"] * 7: it["pix0"] * 7 + 7 * HW].reshape(7, HW)
        off = lambda m: rng.choice([-1.0, 1.0], size=m.shape) * rng.uniform(0.02, 0.3, size=m.shape)  # noqa: E731
        t_rgb.append((im[:3] + off(im[:3])).reshape(-1))
        d = im[3] + off(im[3])
        d[rng.uniform(size=HW) < 0.1] = 0.0
        t_depth.append(d)
        t_sem.append((im[4:] + off(im[4:])).reshape(-1))
    t_rgb, t_depth, t_sem = (np.concatenate(x).astype(np.float32) for x in (t_rgb, t_depth, t_sem))
    T = dict(rgb=torch.from_numpy(t_rgb).cuda(), depth=torch.from_numpy(t_depth).cuda(),
             sem_color=torch.from_numpy(t_sem).cuda())
    ls, grad = raster.loss(cfg, fr, 0, img, T)
    grads = raster.render_bwd(cfg, g, proj, fr, srt, img, grad)
    torch.cuda.synchronize()
    ls_ref, gimg = oracle.loss(views, 3, r["img"], t_rgb, t_depth, None, ssim_lambda=0.2, t_sem=t_sem,
                               sem_ssim_lambda=0.2)
    rel_check(ls.cpu().numpy(), ls_ref, FWD_TOL, name="loss")
    ref = oracle.backward(ocfg, sc, views, gimg)
    mag = oracle.backward(ocfg, sc, views, np.abs(gimg))
    flagged(r["flag"], "pixels")
    bad = flagged(ref["gflag"], "Gaussians touching a flagged pixel", bound=0.15)
    # An entry beyond 1e-3 is one whose pixel terms cancel: it is held to 1e-3 of the sum of
    # their magnitudes (at most 4 such entries per field).
    its = oracle.items(views)
    n_tiles = sum(it["ntx"] * it["nty"] for it in its)
    pre = None
    for name in ("mean", "log_scale", "quat", "opacity", "rgb", "sem"):
        got = grads[name].cpu().numpy()
        m = np.asarray(np.broadcast_to(bad.reshape(-1, *([1] * (got.ndim - 1))), got.shape), bool).reshape(-1)
        kw = dict(mask=m, scale=mag[name] if name in ("rgb", "sem") else None)
        over, err = over_limit(got, ref[name], BWD_TOL, **kw)
        assert len(over) <= 4, (name, len(over))
        for flat in over:
            ix = np.unravel_index(flat, got.shape)
            pre = oracle.preprocess(ocfg, sc, views) if pre is None else pre
            pm = pixel_term_magnitude(ocfg, sc, views, gimg, 7, range(n_tiles), int(ix[0]), name, ix[1:], pre=pre)
            print(f"[semantic colour] {name}{tuple(int(c) for c in ix)}: |d| {err[flat]:.3g}, "
                  f"pixel-term limit {BWD_TOL * pm:.3g}", flush=True)
            assert err[flat] <= BWD_TOL * pm, (name, ix, err[flat], pm)
        kw["mask"] = m | np.isin(np.arange(m.size), over)
        rel_check(got, ref[name], BWD_TOL, name=name, **kw)
    rel_check(grads["pose"].cpu().numpy(), ref["pose"], BWD_TOL, name="pose")
