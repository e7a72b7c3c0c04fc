"""HIP path (through the C ABI) against the FP64 oracle, stage by stage.

Bars: binning (keys, values, ranges) bit-exact; integer projection outputs exact
away from flagged decisions; forward images within 1e-4 relative (per element,
with a floor of 1% of the tensor's rms) away from flagged pixels; gradients within
1e-3 relative away from Gaussians that touch a flagged pixel.
"""
import numpy as np
import pytest

import oracle
from paper_2412_01217_amd import scenes
from tests.helpers import check_with_pixel_terms, flagged, pixel_mask_to_channels, rel_check, targets_from_random

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_TOL = 1e-4
BWD_TOL = 1e-3


def _raster():
    from paper_2412_01217_amd import raster
    return raster


def small_room(n=6000, n_classes=12, W=200, H=136, levels=3, seed=0):
    sc = scenes.room_scene(n=n, n_classes=n_classes, seed=scenes.SEED_SCENE + 10 + seed, log_mu=-3.5)
    views = scenes.room_views(sc, 1, W, H, fx=W / 2, levels=levels, seed=scenes.SEED_VIEWS + 10 + seed)
    return sc, views


CASES = {
    "tiny": lambda: scenes.config_tiny(),
    "room_ragged_3lv": lambda: small_room(),
    "room_two_views": lambda: (lambda sc: (sc, scenes.room_views(sc, 2, 96, 80, levels=2, seed=77)))(
        scenes.room_scene(n=4000, n_classes=5, seed=1077, log_mu=-3.3)),
    # coarse tiles with lists of up to ~3000 blended Gaussians: the reverse pass cuts them
    # into several segments
    "room_long_lists": lambda: (lambda sc: (sc, scenes.room_views(sc, 1, 128, 96, fx=64, levels=3,
                                                                 seed=scenes.SEED_VIEWS + 30)))(
        scenes.room_scene(n=12000, n_classes=6, seed=scenes.SEED_SCENE + 30, log_mu=-3.2)),
}


def _pipeline(sc, views, n_sem, variant=0, split=True, state_capacity=None, fwd_chunk=1, isotropic=False,
              tile=(16, 16), seg_len=0):
    """split: forward with its state (long lists in segments of fwd_chunk seg_len-entry pieces,
    0 = whole lists); state_capacity overrides the capacity the state is sized for;
    isotropic: the primitive of eq. 1-3; tile: the screen tile (width, height); seg_len: list
    entries per segment (0 = 1024)."""
    raster = _raster()
    cfg = raster.config(n_sem, variant=variant, fwd_chunk=fwd_chunk, isotropic=int(isotropic), tile_w=tile[0],
                        tile_h=tile[1], seg_len=seg_len)
    fr = raster.Frame(cfg, views)
    g = raster.to_device(sc)
    proj = raster.preprocess(cfg, g, fr)
    srt = raster.bin_sort(cfg, proj, fr, sc.n, want_keys=True)
    out = None
    if split and state_capacity is not None:
        out = raster.alloc_images(cfg, fr, state_capacity=state_capacity)
    img = raster.render_fwd(cfg, g, proj, fr, srt, out=out, split=split)
    torch.cuda.synchronize()
    return cfg, fr, g, proj, srt, img


def test_item_layout_matches_oracle():
    raster = _raster()
    sc, views = small_room()
    views = views + scenes.room_views(sc, 2, 96, 64, levels=2, seed=9)
    cfg = raster.config(sc.n_classes)
    fr = raster.Frame(cfg, views)
    its = oracle.items(views)
    assert fr.n_items == len(its)
    for a, b in zip(fr.item_list(), its):
        assert (a["W"], a["H"], a["view"], a["level"], a["tile_base"], a["pixel_base"]) == \
               (b["W"], b["H"], b["view"], b["level"], b["tile0"], b["pix0"])


@pytest.mark.parametrize("isotropic", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_preprocess_parity(case, isotropic):
    sc, views = CASES[case]()
    raster = _raster()
    cfg = raster.config(sc.n_classes, isotropic=int(isotropic))
    fr = raster.Frame(cfg, views)
    proj = raster.preprocess(cfg, raster.to_device(sc), fr)
    torch.cuda.synchronize()
    ref = oracle.preprocess(oracle.Config(isotropic=isotropic), sc, views)
    rad = proj["radius"].cpu().numpy()
    rec = proj["rec"].cpu().numpy().reshape(-1, 8).astype(np.float64)
    depth = proj["depth"].cpu().numpy()
    ok = ~flagged(ref["flag"], "projections")
    np.testing.assert_array_equal(rad[ok], ref["radius"][ok])
    vis = ok & (ref["radius"] > 0)
    assert vis.sum() > 100
    m2 = rec[:, 0:2] + rec[:, 2:4]
    rel_check(m2[vis], ref["m2"][vis], 1e-12, floor=1.0, name="mean2d")
    # conic entries relative to the conic's own scale (its larger diagonal entry)
    cscale = np.repeat(np.maximum(np.abs(ref["conic"][vis, 0]), np.abs(ref["conic"][vis, 2]))[:, None], 3, 1)
    rel_check(rec[vis, 4:7], ref["conic"][vis], 1e-6, name="conic", scale=cscale)
    rel_check(rec[vis, 7], ref["opacity"][vis], 2e-7, name="opacity")
    np.testing.assert_array_equal(depth[vis], ref["depth"][vis].astype(np.float32))


def _check_sort(views, n, hi, lo, radius, depth, tile=(16, 16), sort_mode=0):
    raster = _raster()
    cfg = raster.config(0, tile_w=tile[0], tile_h=tile[1], sort_mode=sort_mode)
    fr = raster.Frame(cfg, views)
    E = fr.n_items * n
    rec = np.zeros((E, 8), np.float32)
    rec[:, 0:2] = hi
    rec[:, 2:4] = lo
    rec[:, 4] = rec[:, 6] = 1.0
    rec[:, 7] = 0.5
    proj = dict(rec=torch.from_numpy(rec.reshape(-1)).cuda(), depth=torch.from_numpy(depth).cuda(),
                radius=torch.from_numpy(radius).cuda())
    srt = raster.bin_sort(cfg, proj, fr, n, want_keys=True)
    torch.cuda.synchronize()
    keys, vals, ranges = oracle.sort_stage(views, n, hi, lo, radius, depth, tile_w=tile[0], tile_h=tile[1])
    D = int(srt.n_dup.item())
    assert D == len(keys)
    np.testing.assert_array_equal(srt.keys[:D].cpu().numpy().view(np.uint64), keys)
    np.testing.assert_array_equal(srt.vals[:D].cpu().numpy().view(np.uint32), vals)
    np.testing.assert_array_equal(srt.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges)
    return D


# gs_config.sort_mode: 1 radix passes, 2 bucket path (one counting pass by tile, then per-tile
# depth sorts in LDS)
SORT_MODES = [1, 2]


@pytest.mark.parametrize("sort_mode", SORT_MODES)
@pytest.mark.parametrize("seed,ties", [(1, True), (2, False), (3, True)])
def test_bin_sort_bit_exact_synthetic(seed, ties, sort_mode):
    views = [scenes.identity_view(200, 120, levels=2), scenes.identity_view(64, 48, levels=1),
             scenes.identity_view(100, 70, levels=1)]
    sizes = [(it["W"], it["H"]) for it in oracle.items(views)]
    n = 3000
    hi, lo, radius, depth = scenes.synthetic_projection(sizes, n, seed=5000 + seed, tie_depths=ties)
    assert _check_sort(views, n, hi, lo, radius, depth, sort_mode=sort_mode) > 10000


@pytest.mark.parametrize("sort_mode", SORT_MODES)
def test_bin_sort_bit_exact_on_oracle_projection(sort_mode):
    # inputs: the oracle's own projection of a room scene, rounded to single precision
    sc, views = small_room(n=20000)
    ref = oracle.preprocess(oracle.Config(), sc, views)
    hi = ref["m2"].astype(np.float32)
    lo = (ref["m2"] - hi.astype(np.float64)).astype(np.float32)
    _check_sort(views, sc.n, hi, lo, ref["radius"].astype(np.int32), ref["depth"].astype(np.float32),
                sort_mode=sort_mode)


@pytest.mark.parametrize("sort_mode", SORT_MODES)
@pytest.mark.parametrize("n", [12000, 40000])
def test_bin_sort_bit_exact_long_lists(n, sort_mode):
    """A 64 x 48 image (12 tiles) under thousands of Gaussians of radius up to 40 px, depths
    from a small set (index tie-breaks): tile lists of several thousand entries. The bucket
    path (sort_mode 2) sorts lists of 1025 to 8192 keys by rank in its long-list kernel and
    longer ones (n = 40000: above 16384) with the bitonic network in global memory."""
    views = [scenes.identity_view(64, 48, levels=1)]
    hi, lo, radius, depth = scenes.synthetic_projection([(64, 48)], n, seed=5030 + n, tie_depths=True)
    _check_sort(views, n, hi, lo, radius, depth, sort_mode=sort_mode)
    _, _, ranges = oracle.sort_stage(views, n, hi, lo, radius, depth)
    longest = int((ranges[:, 1] - ranges[:, 0]).max())
    print(f"[long lists] n {n}: longest list {longest}", flush=True)
    assert longest > (4096 if n < 20000 else 16384)


# 256-pixel tiles other than 16 x 16 (the autotuner's tile shapes)
TILE_SHAPES = [(32, 8), (8, 32), (64, 4)]


@pytest.mark.parametrize("sort_mode", SORT_MODES)
@pytest.mark.parametrize("tile", TILE_SHAPES)
def test_bin_sort_bit_exact_tile_shapes(tile, sort_mode):
    views = [scenes.identity_view(200, 120, levels=2), scenes.identity_view(100, 70, levels=1)]
    sizes = [(it["W"], it["H"]) for it in oracle.items(views)]
    hi, lo, radius, depth = scenes.synthetic_projection(sizes, 3000, seed=5020, tie_depths=True)
    assert _check_sort(views, 3000, hi, lo, radius, depth, tile, sort_mode) > 10000
    sc, views = small_room(n=20000)
    ref = oracle.preprocess(oracle.Config(tile_w=tile[0], tile_h=tile[1]), sc, views)
    hi = ref["m2"].astype(np.float32)
    lo = (ref["m2"] - hi.astype(np.float64)).astype(np.float32)
    _check_sort(views, sc.n, hi, lo, ref["radius"].astype(np.int32), ref["depth"].astype(np.float32), tile,
                sort_mode)


@pytest.mark.parametrize("tile", TILE_SHAPES)
def test_preprocess_parity_tile_shapes(tile):
    """A footprint whose rect misses every tile of its item is culled (radius 0): that
    decision depends on the tile shape."""
    sc, views = CASES["room_ragged_3lv"]()
    raster = _raster()
    cfg = raster.config(sc.n_classes, tile_w=tile[0], tile_h=tile[1])
    fr = raster.Frame(cfg, views)
    proj = raster.preprocess(cfg, raster.to_device(sc), fr)
    torch.cuda.synchronize()
    ref = oracle.preprocess(oracle.Config(tile_w=tile[0], tile_h=tile[1]), sc, views)
    ok = ~flagged(ref["flag"], "projections")
    np.testing.assert_array_equal(proj["radius"].cpu().numpy()[ok], ref["radius"][ok])


@pytest.mark.parametrize("variant", ["split", "split_wholewalk", "mfma", "valu"])
@pytest.mark.parametrize("tile", TILE_SHAPES)
@pytest.mark.parametrize("case", ["room_ragged_3lv", "room_long_lists"])
def test_render_parity_tile_shapes(case, tile, variant):
    sc, views = CASES[case]()
    _check_render_fwd(sc, views, *VARIANTS[variant], tile=tile)
    _check_render_bwd(case, *VARIANTS[variant], tile=tile)


@pytest.mark.parametrize("sort_mode", SORT_MODES)
def test_bin_sort_capacity_overflow_reports_status(sort_mode):
    raster = _raster()
    views = [scenes.identity_view(128, 96)]
    n = 500
    hi, lo, radius, depth = scenes.synthetic_projection([(128, 96)], n, seed=5010)
    cfg = raster.config(0, sort_mode=sort_mode)
    fr = raster.Frame(cfg, views)
    rec = np.zeros((n, 8), np.float32)
    rec[:, 0:2], rec[:, 2:4] = hi, lo
    proj = dict(rec=torch.from_numpy(rec.reshape(-1)).cuda(), depth=torch.from_numpy(depth).cuda(),
                radius=torch.from_numpy(radius).cuda())
    s = raster.Sorter(cfg, fr, n, capacity=100).run(proj)
    torch.cuda.synchronize()
    from paper_2412_01217_amd import _lib
    assert int(s.status.item()) == _lib.GS_ERR_CAPACITY
    assert int(s.n_dup.item()) > 100
    # growing the capacity recovers
    s2 = raster.bin_sort(cfg, proj, fr, n)
    assert int(s2.status.item()) == _lib.GS_OK and int(s2.n_dup.item()) == int(s.n_dup.item())


# (render variant, forward with its state, forward chunk): "split_nostate" is the bfloat16
# matrix-core path with every tile list composited whole and the reverse pass's own
# summary pass; with the state, a forward work item walks 1 or 2 segments of 1024 entries
# (longer lists start from the transmittance pre-pass) or the whole list (chunk 0)
VARIANTS = {"valu": (1, False, 1), "mfma": (2, False, 1), "split": (3, True, 1), "split_chunk2": (3, True, 2),
            "split_wholewalk": (3, True, 0), "split_nostate": (3, False, 1)}


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("case", list(CASES))
def test_render_fwd_parity(case, variant):
    sc, views = CASES[case]()
    _check_render_fwd(sc, views, *VARIANTS[variant])


@pytest.mark.parametrize("case", ["room_ragged_3lv", "room_two_views", "room_long_lists"])
def test_render_fwd_parity_isotropic_primitive(case):
    sc, views = CASES[case]()
    _check_render_fwd(sc, views, *VARIANTS["split"], isotropic=True)


def test_render_fwd_state_too_small():
    """A forward state sized for no duplicates cannot hold the long lists' segments; every
    tile is then one item, in the forward and in the reverse pass."""
    sc, views = CASES["room_long_lists"]()
    _check_render_fwd(sc, views, 3, True, state_capacity=0)
    _check_render_bwd("room_long_lists", 3, True, state_capacity=0)
    _check_render_bwd("room_long_lists", 3, True, fwd_chunk=0, state_capacity=0)


@pytest.mark.parametrize("seg_len,fwd_chunk", [(256, 1), (256, 0), (256, 2), (512, 1), (512, 0), (1024, 2)])
def test_render_parity_segment_lengths(seg_len, fwd_chunk):
    """Longer segments of the split lists (the reverse pass's work items and the forward's
    state points): forward and backward against the oracle on lists several segments long."""
    sc, views = CASES["room_long_lists"]()
    _, _, _, _, srt, _ = _pipeline(sc, views, sc.n_classes, 3, True, None, fwd_chunk, seg_len=seg_len)
    lens = srt.ranges.view(-1, 2)[:, 1] - srt.ranges.view(-1, 2)[:, 0]
    longest = int(lens.max().item())
    print(f"[segments] seg_len {seg_len}: longest list {longest}", flush=True)
    assert longest > 2 * seg_len   # lists of three segments and more
    _check_render_fwd(sc, views, 3, True, fwd_chunk, seg_len=seg_len)
    _check_render_bwd("room_long_lists", 3, True, fwd_chunk, seg_len=seg_len)


def _check_render_fwd(sc, views, variant, split, fwd_chunk=1, state_capacity=None, isotropic=False, tile=(16, 16),
                      seg_len=0):
    cfg, fr, g, proj, srt, img = _pipeline(sc, views, sc.n_classes, variant, split, state_capacity, fwd_chunk,
                                           isotropic, tile, seg_len)
    ocfg = oracle.Config(isotropic=isotropic, tile_w=tile[0], tile_h=tile[1])
    ref = oracle.render(ocfg, sc, views)
    # sum_i w_i |f_i|: the magnitude a composited sum with mixed signs is measured against
    mag = oracle.render(ocfg, sc, views, sem=np.abs(sc.sem))["img"]
    its = oracle.items(views)
    K = ref["K"]
    flag = flagged(ref["flag"], "pixels")
    got = img["color"].cpu().numpy()
    mask = pixel_mask_to_channels(flag, its, K)
    for c0, c1, nm in ((0, 3, "rgb"), (3, 4, "depth"), (4, K, "sem")):
        sel = np.zeros(got.shape, bool)
        for it in its:
            HW = it["W"] * it["H"]
            sel[it["pix0"] * K + c0 * HW: it["pix0"] * K + c1 * HW] = True
        rel_check(got[sel], ref["img"][sel], FWD_TOL, mask=mask[sel], name=nm, scale=mag[sel])
    rel_check(img["T"].cpu().numpy(), ref["T"], FWD_TOL, mask=flag, name="T")
    nc = img["n_contrib"].cpu().numpy()
    np.testing.assert_array_equal(nc[~flag], ref["n_contrib"][~flag])


def test_loss_parity_on_shared_images():
    raster = _raster()
    sc, views = small_room(n_classes=9)
    cfg = raster.config(9)
    fr = raster.Frame(cfg, views)
    K = 13
    img = scenes.random_image(fr.n_pixels, K, seed=5101)
    t_rgb, t_depth, t_lab = targets_from_random(views, 9, seed=4001)
    w = (0.8, 1.1, 0.6)
    ls_ref, g_ref = oracle.loss(views, 9, img, t_rgb, t_depth, t_lab, w=w)
    T = dict(rgb=torch.from_numpy(t_rgb).cuda(), depth=torch.from_numpy(t_depth).cuda(),
             label=torch.from_numpy(t_lab).cuda())
    rendered = dict(color=torch.from_numpy(img).cuda())
    ls, grad = raster.loss(cfg, fr, 9, rendered, T, w=w)
    torch.cuda.synchronize()
    rel_check(ls.cpu().numpy(), ls_ref, 1e-5, name="loss")
    d = img.astype(np.float64)
    near_kink = np.zeros(d.shape, bool)     # |R - R_gt| tiny: the L1 sign may differ in FP32
    rel_check(grad["color"].cpu().numpy(), g_ref, 1e-5, mask=near_kink, name="dloss/dimg")


SSIM_VIEWS = {
    # 200 x 136 with 3 levels: several 32 x 32 SSIM tiles per level with ragged tails, and a
    # 50 x 34 level barely wider than one tile
    "room": lambda: small_room(n_classes=9)[1],
    # images smaller than the 11 x 11 window next to a larger one
    "tiny_items": lambda: [scenes.identity_view(8, 6, levels=1), scenes.identity_view(72, 40, levels=2),
                           scenes.identity_view(4, 4, levels=2)],
}


@pytest.mark.parametrize("lam", [0.2, 1.0])
@pytest.mark.parametrize("case", list(SSIM_VIEWS))
def test_loss_parity_with_ssim(case, lam):
    raster = _raster()
    views = SSIM_VIEWS[case]()
    cfg = raster.config(9)
    cfg.ssim_lambda = lam
    fr = raster.Frame(cfg, views)
    K = 13
    img = scenes.random_image(fr.n_pixels, K, seed=5102)
    t_rgb, t_depth, t_lab = targets_from_random(views, 9, seed=4002)
    w = (0.8, 1.1, 0.6)
    ls_ref, g_ref = oracle.loss(views, 9, img, t_rgb, t_depth, t_lab, w=w, ssim_lambda=lam)
    T = dict(rgb=torch.from_numpy(t_rgb).cuda(), depth=torch.from_numpy(t_depth).cuda(),
             label=torch.from_numpy(t_lab).cuda())
    rendered = dict(color=torch.from_numpy(img).cuda())
    ls, grad = raster.loss(cfg, fr, 9, rendered, T, w=w)
    torch.cuda.synchronize()
    rel_check(ls.cpu().numpy(), ls_ref, FWD_TOL, name="loss")
    rel_check(grad["color"].cpu().numpy(), g_ref, BWD_TOL, name="dloss/dimg")
    # the same call again: the workspace's slots are cleared by every call (the slot sums
    # are float atomics, so only their order, not their content, may differ)
    ls2, _ = raster.loss(cfg, fr, 9, rendered, T, w=w)
    torch.cuda.synchronize()
    np.testing.assert_allclose(ls2.cpu().numpy(), ls.cpu().numpy(), rtol=1e-6)


def _shared_grad_image(fr, K, seed):
    return scenes.random_image(fr.n_pixels, K, seed=seed, scale=1e-3)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("case", list(CASES))
def test_render_bwd_parity(case, variant):
    _check_render_bwd(case, *VARIANTS[variant])


@pytest.mark.parametrize("case", ["room_ragged_3lv", "room_two_views", "room_long_lists"])
def test_render_bwd_parity_isotropic_primitive(case):
    _check_render_bwd(case, *VARIANTS["split"], isotropic=True)


@pytest.mark.parametrize("split", [True, False])
def test_render_bwd_single_item_fallback(split):
    """A workspace sized without the duplicate capacity cannot hold every segment of the
    long lists; the reverse pass then takes each tile as one work item."""
    _check_render_bwd("room_long_lists", 3, split, small_workspace=True)


def _check_render_bwd(case, variant, split, fwd_chunk=1, small_workspace=False, state_capacity=None,
                      isotropic=False, tile=(16, 16), seg_len=0):
    sc, views = CASES[case]()
    cfg, fr, g, proj, srt, img = _pipeline(sc, views, sc.n_classes, variant, split, state_capacity, fwd_chunk,
                                           isotropic, tile, seg_len)
    ocfg = oracle.Config(isotropic=isotropic, tile_w=tile[0], tile_h=tile[1])
    raster = _raster()
    ws = None
    if small_workspace:
        nb = raster.workspace_bytes(raster.L.GS_WS_RENDER_BWD, cfg, fr, sc.n, 0)
        assert nb < raster.workspace_bytes(raster.L.GS_WS_RENDER_BWD, cfg, fr, sc.n, srt.capacity)
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    K = 4 + sc.n_classes
    gimg = _shared_grad_image(fr, K, seed=5200)
    # pixels whose forward decisions sit within rounding of a threshold get no upstream
    # gradient, so they cannot contribute to any parameter's gradient on either side
    r = oracle.render(ocfg, sc, views)
    gimg[pixel_mask_to_channels(flagged(r["flag"], "pixels"), oracle.items(views), K)] = 0.0
    grads = raster.render_bwd(cfg, g, proj, fr, srt, img, dict(color=torch.from_numpy(gimg).cuda()), ws=ws)
    torch.cuda.synchronize()
    ref = oracle.backward(ocfg, sc, views, gimg)
    # features enter linearly: sum_p w |g_p| bounds their gradients' terms
    mag = oracle.backward(ocfg, sc, views, np.abs(gimg))
    pre = None
    for name in ("mean", "log_scale", "quat", "opacity", "rgb", "sem"):
        got = grads[name].cpu().numpy()
        if name in ("rgb", "sem"):
            rel_check(got, ref[name], BWD_TOL, name=name, scale=mag[name])
        else:   # an entry whose pixel terms cancel is held to 1e-3 of their magnitudes (at most 4)
            pre = check_with_pixel_terms(got, ref[name], BWD_TOL, name, ocfg, sc, views, gimg.astype(np.float64), K,
                                         pre=pre)
    if isotropic:           # eq. 1-3 use one scale and no rotation
        assert not grads["quat"].any() and not grads["log_scale"][:, 1:].any()
    rel_check(grads["pose"].cpu().numpy(), ref["pose"], BWD_TOL, name="pose")


@pytest.mark.parametrize("lam", [0.0, 0.2])
def test_end_to_end_tiny_loss_and_gradients(lam):
    sc, views = scenes.config_tiny()
    cfg, fr, g, proj, srt, img = _pipeline(sc, views, 8)
    cfg.ssim_lambda = lam
    raster = _raster()
    t_rgb, t_depth, t_lab = targets_from_random(views, 8, seed=4000, invalid_frac=0.0)
    T = dict(rgb=torch.from_numpy(t_rgb).cuda(), depth=torch.from_numpy(t_depth).cuda(),
             label=torch.from_numpy(t_lab).cuda())
    ls, grad = raster.loss(cfg, fr, 8, img, T)
    grads = raster.render_bwd(cfg, g, proj, fr, srt, img, grad)
    torch.cuda.synchronize()
    r = oracle.render(oracle.Config(), sc, views)
    ls_ref, gimg = oracle.loss(views, 8, r["img"], t_rgb, t_depth, t_lab, ssim_lambda=lam)
    rel_check(ls.cpu().numpy(), ls_ref, 1e-4, name="loss")
    ref = oracle.backward(oracle.Config(), sc, views, gimg)
    # features enter linearly: sum_p w |g_p| bounds their gradients' terms
    mag = oracle.backward(oracle.Config(), sc, views, np.abs(gimg))
    flagged(r["flag"], "pixels")
    # every contributor of a flagged pixel (4 pixels here reach about 9 % of the Gaussians)
    bad = flagged(ref["gflag"], "Gaussians touching a flagged pixel", bound=0.15)
    for name in ("mean", "log_scale", "quat", "opacity", "rgb", "sem"):
        got = grads[name].cpu().numpy()
        m = np.broadcast_to(bad.reshape(-1, *([1] * (got.ndim - 1))), got.shape)
        rel_check(got, ref[name], BWD_TOL, mask=m, name=name, scale=mag[name] if name in ("rgb", "sem") else None)


def test_empty_and_culled_scenes():
    raster = _raster()
    views = [scenes.identity_view(40, 24, levels=1)]
    # all Gaussians behind the camera
    sc = scenes.tiny_scene(n=50, n_classes=3)
    sc.mean[:, 2] = -1.0
    cfg, fr, g, proj, srt, img = _pipeline(sc, views, 3)
    assert int(srt.n_dup.item()) == 0
    np.testing.assert_array_equal(img["color"].cpu().numpy(), 0)
    np.testing.assert_array_equal(img["T"].cpu().numpy(), 1)
    gimg = _shared_grad_image(fr, 7, seed=5201)
    grads = raster.render_bwd(cfg, g, proj, fr, srt, img, dict(color=torch.from_numpy(gimg).cuda()))
    torch.cuda.synchronize()
    for k in ("mean", "rgb", "sem", "pose"):
        np.testing.assert_array_equal(grads[k].cpu().numpy(), 0)
    # a zero quaternion is culled rather than producing NaN
    sc2 = scenes.tiny_scene(n=30, n_classes=3)
    sc2.quat[0] = 0.0
    cfg, fr, g, proj, srt, img = _pipeline(sc2, views, 3)
    assert int(proj["radius"][0].item()) == 0
    assert np.isfinite(img["color"].cpu().numpy()).all()


def test_downsample_parity():
    raster = _raster()
    views = [scenes.identity_view(64, 48, levels=3), scenes.identity_view(40, 24, levels=2)]
    cfg = raster.config(5)
    fr = raster.Frame(cfg, views)
    K = 9
    img = scenes.random_image(fr.n_pixels, K, seed=5300)
    # positive depths with some missing
    its = oracle.items(views)
    for it in its:
        HW = it["W"] * it["H"]
        d = img[it["pix0"] * K + 3 * HW: it["pix0"] * K + 4 * HW]
        d[:] = np.where(np.abs(d) < 0.3, 0.0, np.abs(d))
    ref, lab_ref = oracle.downsample(views, 5, img)
    t = torch.from_numpy(img.copy()).cuda()
    lab = torch.empty(fr.n_pixels, dtype=torch.int32, device="cuda")
    raster.downsample(fr, K, t, lab)
    torch.cuda.synchronize()
    rel_check(t.cpu().numpy(), ref, 2e-5, name="pyramid")
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref)
