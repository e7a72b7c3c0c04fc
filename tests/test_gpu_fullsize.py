"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

- the whole bin sort, bit-exact, against the oracle's sort stage run on the GPU's own
  single-precision projections;
- the forward on every tile (room) or on sampled tiles (the 8-view batch: the longest lists
  and random ones; the oracle renders only those tiles), and every gradient from an upstream
  gradient confined to sampled tiles (the oracle differentiates only those tiles);
- the learned batch (52 classes through the head, its decode fused into the loss): the
  forward on sampled tiles, the embedding and geometry gradients from the step's own loss
  gradient confined to them;
- the loss with the SSIM term over the full room pyramid.
"""
import ctypes

import numpy as np
import pytest

import oracle
from tests.helpers import flagged, over_limit, pixel_mask_to_channels, pixel_term_magnitude, rel_check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_TOL = 1e-4
BWD_TOL = 1e-3


def _workload(name, ssim_lambda=0.0):
    import bench
    from paper_2412_01217_amd import autotune, scenes
    from paper_2412_01217_amd.step import MappingStep
    if name == "room":                     # the headline workload, default launch
        sc, views = scenes.config_room()
        st, tg = bench.plain_step(sc, views, "cuda:0", ssim_lambda=ssim_lambda)
    else:                                  # the 8-view batch, in the autotuner's configuration
        sc, views = scenes.config_batch()
        st, tg = bench.plain_step(sc, views, "cuda:0")

        def make(cfg):
            return MappingStep(cfg, autotune.frame_for(cfg, st.frame), st.g, tg, sc.n_classes)
        autotune.tune(make, st.cfg, st.frame, sc.n)
        st = make(st.cfg)
    return sc, views, st, tg


def _tile_pixels(its, mask, tile=(16, 16)):
    """Per pixel of the concatenated items: does its tile belong to the sample."""
    sel = []
    for it in its:
        v, u = np.mgrid[0:it["H"], 0:it["W"]]
        t = it["tile0"] + (v // tile[1]) * it["ntx"] + (u // tile[0])
        sel.append(mask[t.reshape(-1)] != 0)
    return np.concatenate(sel)


@pytest.mark.parametrize("name", ["room", "batch"])
def test_full_size_sort_and_sampled_tiles(name):
    from paper_2412_01217_amd import raster
    sc, views, st, tg = _workload(name)
    st.run()
    torch.cuda.synchronize()
    assert not st.overflowed()
    # the whole sort, on the GPU's own projections
    rec = st.proj["rec"].cpu().numpy().reshape(-1, 8)
    radius = st.proj["radius"].cpu().numpy()
    depth = st.proj["depth"].cpu().numpy()
    tile = st.frame.tile                   # the launch's tile shape (the autotuner may pick another)
    print(f"[full size] {name}: tile {tile}, variant {st.cfg.variant}, fwd_chunk {st.cfg.fwd_chunk}", flush=True)
    keys, vals, ranges = oracle.sort_stage(views, sc.n, rec[:, 0:2], rec[:, 2:4], radius, depth, tile_w=tile[0],
                                           tile_h=tile[1])
    D = int(st.sorter.n_dup.item())
    assert D == len(vals) and D > 100_000
    np.testing.assert_array_equal(st.sorter.vals[:D].cpu().numpy().view(np.uint32), vals)
    np.testing.assert_array_equal(st.sorter.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges)
    # both sort methods (gs_config.sort_mode 1: radix passes, 2: bucket path) on the same
    # projections
    for mode in (1, 2):
        cfg = type(st.cfg)()
        ctypes.memmove(ctypes.byref(cfg), ctypes.byref(st.cfg), ctypes.sizeof(cfg))
        cfg.sort_mode = mode
        other = raster.Sorter(cfg, st.frame, sc.n, st.sorter.capacity).run(st.proj)
        torch.cuda.synchronize()
        print(f"[full size] {name}: sort_mode {mode}", flush=True)
        assert int(other.status.item()) == 0 and int(other.n_dup.item()) == D
        np.testing.assert_array_equal(other.vals[:D].cpu().numpy().view(np.uint32), vals)
        np.testing.assert_array_equal(other.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges)
        del other

    # sampled tiles: the longest lists and random ones
    its = oracle.items(views, *tile)
    ntiles = len(ranges)
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    rng = np.random.default_rng(7700)
    n_rand = 20 if name == "room" else 8
    pick = set(np.argsort(-lens)[:4].tolist()) | set(rng.choice(ntiles, n_rand, replace=False).tolist())
    mask = np.zeros(ntiles, np.uint8)
    mask[sorted(pick)] = 1
    ocfg = oracle.Config(tile_w=tile[0], tile_h=tile[1])
    # the room is compared on every tile (the oracle renders it whole in a few seconds)
    fmask = None if name == "room" else mask
    ref = oracle.render(ocfg, sc, views, tile_mask=fmask)
    mag = oracle.render(ocfg, sc, views, sem=np.abs(sc.sem), tile_mask=fmask)["img"]
    K = ref["K"]
    sel = np.ones(len(ref["T"]), bool) if fmask is None else _tile_pixels(its, mask, tile)
    flag = flagged(ref["flag"][sel], "pixels compared")
    keep_px = sel.copy()
    keep_px[np.flatnonzero(sel)[flag]] = False
    keep = pixel_mask_to_channels(keep_px, its, K)
    got = st.img["color"].cpu().numpy()
    rel_check(got, ref["img"], FWD_TOL, mask=~keep, name="image", scale=mag)
    rel_check(st.img["T"].cpu().numpy(), ref["T"], FWD_TOL, mask=~keep_px, name="T")
    nc = st.img["n_contrib"].cpu().numpy()
    np.testing.assert_array_equal(nc[keep_px], ref["n_contrib"][keep_px])

    # backward from an upstream gradient on the sampled tiles only
    keep = pixel_mask_to_channels(keep_px & _tile_pixels(its, mask, tile), its, K)
    gimg = (rng.normal(size=got.shape) * 1e-3).astype(np.float32)
    gimg[~keep] = 0.0
    grads = raster.render_bwd(st.cfg, st.g, st.proj, st.frame, st.sorter, st.img,
                              dict(color=torch.from_numpy(gimg).cuda()), ws=st.bwd_ws)
    torch.cuda.synchronize()
    ob = oracle.backward(ocfg, sc, views, gimg.astype(np.float64), tile_mask=mask)
    om = oracle.backward(ocfg, sc, views, np.abs(gimg.astype(np.float64)), tile_mask=mask)
    # a Gaussian's geometric gradient sums the sampled tiles' contributions, which may cancel:
    # its error is measured against the sum of their magnitudes (one tile at a time)
    geo = ("mean", "log_scale", "quat", "opacity")
    per_tile = {k: np.zeros_like(ob[k]) for k in geo}
    for t in sorted(pick):
        m1 = np.zeros_like(mask)
        m1[t] = 1
        o1 = oracle.backward(ocfg, sc, views, gimg.astype(np.float64), tile_mask=m1)
        for k in geo:
            per_tile[k] += np.abs(o1[k])
    # Within a tile the pixels on either side of a footprint's centre contribute with opposite
    # signs as well; at full size (600k-4M Gaussians) the few gradients dominated by that are
    # held to the same 1e-3 against 5 % of the rms as a floor, and every gradient field to a
    # relative L2 error of 1e-5.
    bad = ob["gflag"] != 0
    for k in ("mean", "log_scale", "quat", "opacity", "rgb", "sem"):
        g = grads[k].cpu().numpy()
        m = np.broadcast_to(bad.reshape(-1, *([1] * (g.ndim - 1))), g.shape)
        feat = k in ("rgb", "sem")
        res = rel_check(g, ob[k], BWD_TOL, mask=m, name=k, scale=om[k] if feat else per_tile[k],
                        floor=0.01 if feat else 0.05)
        assert res["l2"] < 1e-5, (k, res)
    rel_check(grads["pose"].cpu().numpy(), ob["pose"], BWD_TOL, name="pose")


def test_full_size_loss_with_ssim_on_the_room_pyramid():
    sc, views, st, tg = _workload("room", ssim_lambda=0.2)
    st.run()
    torch.cuda.synchronize()
    img = st.img["color"].cpu().numpy()
    ls_ref, g_ref = oracle.loss(views, sc.n_classes, img, tg["rgb"].cpu().numpy(), tg["depth"].cpu().numpy(),
                                tg["label"].cpu().numpy(), ssim_lambda=0.2)
    rel_check(st.loss.view(-1, 3).cpu().numpy(), ls_ref, FWD_TOL, name="loss")
    # a colour gradient is (1 - lambda) sign(d) / (3HW) plus the SSIM term; where the two
    # nearly cancel, the sum is measured against the L1 term's size
    K = 4 + sc.n_classes
    scale = np.zeros(len(g_ref))
    for it in oracle.items(views):
        HW = it["W"] * it["H"]
        scale[it["pix0"] * K: it["pix0"] * K + 3 * HW] = (1 - 0.2) / (3 * HW)
    rel_check(st.grad["color"].cpu().numpy(), g_ref, BWD_TOL, name="dloss/dimg", scale=scale)


def test_full_size_learned_batch_sampled_tiles():
    """The learned 8-view batch (500k Gaussians, 52 classes through the head) in the launch
    the benchmark times: its whole step runs (decode fused into the loss); the composited
    rgb, depth and embedding are compared on sampled tiles, and the gradients of every
    Gaussian parameter (the embedding's included) from an upstream gradient confined to
    them."""
    import bench
    from paper_2412_01217_amd import raster, scenes
    sc, views = scenes.config_learned()
    rng = np.random.default_rng(7710)
    w = scenes.head_weights(52, seed=6030)
    head = dict(W1=torch.from_numpy(w["W1"].view(np.int16).copy()).cuda(), b1=torch.from_numpy(w["b1"]).cuda(),
                W2=torch.from_numpy(w["W2"].view(np.int16).copy()).cuda(), b2=torch.from_numpy(w["b2"]).cuda())
    cfg_p = raster.config(52)
    tg = bench.make_targets(cfg_p, raster.Frame(cfg_p, views), sc, "cuda:0")
    st = bench.learned_step(sc, views, head, "cuda:0", tg)
    st.run()
    torch.cuda.synchronize()
    assert not st.overflowed()
    assert np.isfinite(st.loss.cpu().numpy()).all()
    its = oracle.items(views)
    ranges = st.sorter.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    ntiles = len(ranges)
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    pick = set(np.argsort(-lens)[:4].tolist()) | set(rng.choice(ntiles, 8, replace=False).tolist())
    mask = np.zeros(ntiles, np.uint8)
    mask[sorted(pick)] = 1
    emb = scenes.bf16_bits_to_f32(sc.emb).astype(np.float64)
    ocfg = oracle.Config()
    ref = oracle.render(ocfg, sc, views, sem=emb, tile_mask=mask)
    mag = oracle.render(ocfg, sc, views, sem=np.abs(emb), tile_mask=mask)["img"]
    K = 20
    sel = _tile_pixels(its, mask)
    flag = flagged(ref["flag"][sel], "sampled pixels")
    keep_px = sel.copy()
    keep_px[np.flatnonzero(sel)[flag]] = False
    keep = pixel_mask_to_channels(keep_px, its, K)
    got = st.img["color"].cpu().numpy()
    rel_check(got, ref["img"], FWD_TOL, mask=~keep, name="rgb/depth/E", scale=mag)
    nc = st.img["n_contrib"].cpu().numpy()
    np.testing.assert_array_equal(nc[keep_px], ref["n_contrib"][keep_px])
    gimg = (rng.normal(size=got.shape) * 1e-3).astype(np.float32)
    gimg[~keep] = 0.0
    grads = raster.render_bwd(st.cfg, st.g, st.proj, st.frame, st.sorter, st.img,
                              dict(color=torch.from_numpy(gimg).cuda(), logits=None), ws=st.bwd_ws)
    torch.cuda.synchronize()
    g64 = gimg.astype(np.float64)
    ob = oracle.backward(ocfg, sc, views, g64, sem=emb, tile_mask=mask)
    om = oracle.backward(ocfg, sc, views, np.abs(g64), sem=emb, tile_mask=mask)
    geo = ("mean", "log_scale", "quat", "opacity")
    per_tile = {k: np.zeros_like(ob[k]) for k in geo}
    for t in sorted(pick):
        m1 = np.zeros_like(mask)
        m1[t] = 1
        o1 = oracle.backward(ocfg, sc, views, g64, sem=emb, tile_mask=m1)
        for k in geo:
            per_tile[k] += np.abs(o1[k])
    # as for the plain workloads: Gaussians that also reach a flagged pixel are left out, and
    # the geometric gradients are held to 1e-3 of max(|ref|, the sum of the per-tile
    # magnitudes, 5 % of the rms)
    bad = flagged(ob["gflag"], "Gaussians touching a flagged pixel", bound=0.01)
    # an entry beyond that limit is one whose pixel terms cancel within a tile: it is held to
    # 1e-3 of the sum of its pixel terms' magnitudes (at most 4 such entries per field)
    pre = None
    for k, ko in (("mean", "mean"), ("log_scale", "log_scale"), ("quat", "quat"), ("opacity", "opacity"),
                  ("rgb", "rgb"), ("emb", "sem")):
        g = grads[k].cpu().numpy()
        m = np.broadcast_to(bad.reshape(-1, *([1] * (g.ndim - 1))), g.shape)
        feat = k in ("rgb", "emb")
        lim_kw = dict(mask=m, scale=om[ko] if feat else per_tile[k], floor=0.01 if feat else 0.05)
        over, err = over_limit(g, ob[ko], BWD_TOL, **lim_kw)
        assert len(over) <= 4, (k, len(over))
        for flat in over:
            i, comp = np.unravel_index(flat, g.shape)[0], np.unravel_index(flat, g.shape)[1:]
            pre = oracle.preprocess(ocfg, sc, views) if pre is None else pre
            mag = pixel_term_magnitude(ocfg, sc, views, g64, K, sorted(pick), int(i), ko, comp, sem=emb, pre=pre)
            print(f"[full size] {k}{(int(i),) + tuple(int(c) for c in comp)}: |d| {err[flat]:.3g}, "
                  f"pixel-term limit {BWD_TOL * mag:.3g}", flush=True)
            assert err[flat] <= BWD_TOL * mag, (k, int(i), comp, err[flat], mag)
        res = rel_check(g, ob[ko], BWD_TOL, name=k, **dict(lim_kw, mask=np.asarray(m, bool).copy().reshape(-1) |
                                                              np.isin(np.arange(g.size), over)))
        assert res["l2"] < 1e-5, (k, res)
    rel_check(grads["pose"].cpu().numpy(), ob["pose"], BWD_TOL, name="pose")
