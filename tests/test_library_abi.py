"""CPU-side checks of the C ABI: the library loads, exports every symbol gs.h
declares, and its host-only helpers (no GPU needed) behave."""
import ctypes
import os
import re

import pytest

from paper_2412_01217_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gs.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(gs_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(L.Config) == 76
    assert ctypes.sizeof(L.Targets) == 32
    assert ctypes.sizeof(L.Images) == 56
    assert ctypes.sizeof(L.View) == 56
    assert ctypes.sizeof(L.Item) == 56
    assert ctypes.sizeof(L.Gaussians) == 64


def test_defaults_and_status_strings():
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    assert (c.tile_w, c.tile_h) == (16, 16)
    assert c.alpha_min == pytest.approx(1 / 255) and c.alpha_max == pytest.approx(0.99)
    assert c.t_min == pytest.approx(1e-4) and c.z_near == pytest.approx(0.2)
    assert (c.variant, c.tile_order, c.fwd_chunk, c.ssim_lambda, c.isotropic, c.view_features) == (0, 0, 0, 0.0, 0, 0)
    assert c.sem_ssim_lambda == 0.0 and c.seg_len == 0 and c.sort_mode == 0
    assert lib.gs_status_string(L.GS_ERR_CAPACITY) == b"duplicate capacity exceeded"
    assert lib.gs_version() > 0


def _make(levels, W, H, K=(100.0, 100.0, 64.0, 48.0)):
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    nv = len(levels)
    V = (L.View * nv)()
    items = (L.Item * sum(levels))()
    Wa = (ctypes.c_int32 * nv)(*W)
    Ha = (ctypes.c_int32 * nv)(*H)
    Ka = (ctypes.c_float * (4 * nv))(*(list(K) * nv))
    La = (ctypes.c_int32 * nv)(*levels)
    npx = ctypes.c_int64()
    nt = ctypes.c_int32()
    r = lib.gs_make_items(ctypes.byref(c), nv, V, Wa, Ha, Ka, La, items, ctypes.byref(npx), ctypes.byref(nt))
    return r, V, items, npx.value, nt.value


def test_make_items_pyramid_layout():
    r, V, items, npx, nt = _make([3, 1], [1200, 64], [680, 48], K=(600.0, 600.0, 600.0, 340.0))
    assert r == 4
    assert [(it.W, it.H, it.level) for it in items] == [(1200, 680, 0), (600, 340, 1), (300, 170, 2), (64, 48, 0)]
    assert items[2].fx == 150.0 and items[2].cx == 150.0 and items[1].cy == 170.0
    assert items[1].tile_base == 75 * 43 and items[1].pixel_base == 1200 * 680
    assert npx == 1200 * 680 + 600 * 340 + 300 * 170 + 64 * 48
    assert nt == 75 * 43 + 38 * 22 + 19 * 11 + 4 * 3
    assert (V[0].item_first, V[0].item_count, V[1].item_first) == (0, 3, 3)


def test_make_items_rejects_indivisible_pyramid():
    r, *_ = _make([3], [100], [70])
    assert r == L.GS_ERR_INVALID_ARG


def test_entry_points_reject_bad_arguments_on_host():
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    c.tile_w = 8
    g = L.Gaussians()
    p = L.Projected()
    assert lib.gs_preprocess(ctypes.byref(c), ctypes.byref(g), None, 0, None, 0, ctypes.byref(p), None) == \
        L.GS_ERR_INVALID_ARG
    lib.gs_config_default(ctypes.byref(c))
    c.n_sem = 61
    b = ctypes.c_size_t()
    assert lib.gs_workspace_size(L.GS_WS_BIN_SORT, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == \
        L.GS_ERR_INVALID_ARG
    lib.gs_config_default(ctypes.byref(c))
    assert lib.gs_workspace_size(L.GS_WS_BIN_SORT, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == 0
    assert b.value > 0
    # workspace too small is reported before any launch
    g.n = 10
    assert lib.gs_bin_sort(ctypes.byref(c), ctypes.byref(p), ctypes.c_void_p(16), 1, 10, 4, 100,
                           ctypes.c_void_p(16), 1, None, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None,
                           None) in (L.GS_ERR_INVALID_ARG, L.GS_ERR_WORKSPACE)


def test_forward_state_size_and_host_check():
    """The forward state grows with the duplicate capacity and the channel count; a state
    buffer too small for even one item per tile is refused before any launch."""
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    c.n_sem = 12
    b0, b1, b2 = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.gs_workspace_size(L.GS_WS_RENDER_STATE, ctypes.byref(c), 3, 100, 40, 0, 0, ctypes.byref(b0)) == 0
    assert lib.gs_workspace_size(L.GS_WS_RENDER_STATE, ctypes.byref(c), 3, 100, 40, 10000, 0, ctypes.byref(b1)) == 0
    c.n_sem = 20
    assert lib.gs_workspace_size(L.GS_WS_RENDER_STATE, ctypes.byref(c), 3, 100, 40, 10000, 0, ctypes.byref(b2)) == 0
    # one slot per tile (and one spare) at capacity 0, ceil(10000 / 1024) = 10 more segments
    # of the default length at 10000 duplicates
    slot = 256 * 4 * (4 + 12 + 3)
    assert b0.value >= 41 * slot
    assert 10 * slot <= b1.value - b0.value < 11 * slot
    assert b2.value > b1.value
    # sized for the configured segment length: 40 more at 256 entries, 3 more at 4096
    for seg, more in ((256, 40), (4096, 3)):
        c.n_sem, c.seg_len = 12, seg
        bs = ctypes.c_size_t()
        assert lib.gs_workspace_size(L.GS_WS_RENDER_STATE, ctypes.byref(c), 3, 100, 40, 10000, 0, ctypes.byref(bs)) == 0
        assert more * slot <= bs.value - b0.value < (more + 1) * slot, seg
    c.seg_len = 0
    c.n_sem = 12
    fake = ctypes.c_void_p(256)
    g = L.Gaussians(10, fake, fake, fake, fake, fake, fake, None)
    p = L.Projected(fake, fake, fake)
    im = L.Images(fake, fake, fake, None, 0, fake, b0.value - 1)
    assert lib.gs_render_fwd(ctypes.byref(c), ctypes.byref(g), ctypes.byref(p), fake, 1, 40, fake, fake, None,
                             ctypes.byref(im), None) == L.GS_ERR_WORKSPACE


def test_config_rejects_out_of_range_forward_chunk():
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    b = ctypes.c_size_t()
    for bad in (-1, 65536):
        c.fwd_chunk = bad
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == \
            L.GS_ERR_INVALID_ARG
    for good in (0, 1, 65535):
        c.fwd_chunk = good
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == 0


def test_config_segment_length():
    # split lists' segments: 0 (1024 entries) or a multiple of 32 from 256 to 2^20; the
    # reverse pass's workspace holds more segments, so is larger, for shorter ones
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    b = ctypes.c_size_t()
    for bad in (-32, 32, 224, 250, 1000, (1 << 20) + 32):
        c.seg_len = bad
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == \
            L.GS_ERR_INVALID_ARG, bad
    for good in (0, 256, 288, 1024, 4096, 1 << 20):
        c.seg_len = good
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == 0, good
    sizes = []
    for seg in (256, 1024, 4096):
        c.seg_len = seg
        assert lib.gs_workspace_size(L.GS_WS_RENDER_BWD, ctypes.byref(c), 3, 1000, 40, 10 ** 6, 100,
                                     ctypes.byref(b)) == 0
        sizes.append(b.value)
    assert sizes[0] > sizes[1] > sizes[2]


def test_config_sort_mode_and_workspace():
    # 0 automatic, 1 radix passes, 2 bucket path; the bin-sort workspace covers both methods:
    # at least the bucket path's 8-byte scatter keys
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    b = ctypes.c_size_t()
    for bad in (-1, 3):
        c.sort_mode = bad
        assert lib.gs_workspace_size(L.GS_WS_BIN_SORT, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == \
            L.GS_ERR_INVALID_ARG, bad
    sizes = []
    for good in (0, 1, 2):
        c.sort_mode = good
        assert lib.gs_workspace_size(L.GS_WS_BIN_SORT, ctypes.byref(c), 3, 1000, 50000, 10 ** 6, 100,
                                     ctypes.byref(b)) == 0
        sizes.append(b.value)
    assert sizes[0] == sizes[1] == sizes[2] >= 8 * 10 ** 6


def test_config_rejects_ssim_weight_outside_unit_interval():
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    b = ctypes.c_size_t()
    for bad in (-0.1, 1.5, float("nan")):
        c.ssim_lambda = bad
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == \
            L.GS_ERR_INVALID_ARG
    for good in (0.0, 0.2, 1.0):
        c.ssim_lambda = good
        assert lib.gs_workspace_size(L.GS_WS_LOSS, ctypes.byref(c), 1, 10, 4, 100, 100, ctypes.byref(b)) == 0


def test_mapping_update_structs_and_argument_checks():
    lib = L.lib()
    assert ctypes.sizeof(L.ParamArrays) == 48 and ctypes.sizeof(L.AdamConfig) == 44
    fake = ctypes.c_void_p(256)
    p = L.ParamArrays(fake, fake, fake, fake, fake, None)
    g = L.Grads(*([fake] * 12))

    def hp(**kw):
        h = L.AdamConfig(1e-3, 1e-3, 1e-3, 1e-2, 1e-2, 0.0, 1e-3, 1e-3, 0.9, 0.999, 1e-8)
        for k, val in kw.items():
            setattr(h, k, val)
        return h
    call = lambda n, n_sem, h, step, sem=None: lib.gs_gaussians_adam(  # noqa: E731
        n, n_sem, ctypes.byref(p if sem is None else sem), ctypes.byref(g), ctypes.byref(p), ctypes.byref(p),
        ctypes.byref(h), step, None)
    assert call(0, 0, hp(), 1) == L.GS_OK                              # nothing to update: no launch
    for bad in (dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0), dict(lr_mean=-1.0), dict(lr_phi=float("inf"))):
        assert call(0, 0, hp(**bad), 1) == L.GS_ERR_INVALID_ARG, bad
    assert call(0, 0, hp(), 0) == L.GS_ERR_INVALID_ARG                 # steps count from 1
    assert call(-1, 0, hp(), 1) == L.GS_ERR_INVALID_ARG
    # a semantic group with a nonzero rate needs its arrays
    assert call(5, 3, hp(lr_sem=1e-2), 1) == L.GS_ERR_INVALID_ARG
    assert lib.gs_pose_adam(None, 0, None, None, None, ctypes.byref(hp()), 1, None) == L.GS_OK
    assert lib.gs_pose_adam(None, 2, fake, fake, fake, ctypes.byref(hp()), 1, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_pose_adam(fake, 2, fake, fake, fake, ctypes.byref(hp()), 0, None) == L.GS_ERR_INVALID_ARG


def test_sh_struct_and_argument_checks():
    lib = L.lib()
    assert ctypes.sizeof(L.SH) == 24
    fake = ctypes.c_void_p(256)
    g = L.Gaussians(10, fake, fake, fake, fake, fake, fake, None)
    ok = L.SH(3, 1, fake, fake)
    assert lib.gs_sh_features(4, ctypes.byref(g), ctypes.byref(ok), fake, 0, fake, fake, None) == L.GS_OK
    for bad in (L.SH(4, 0, fake, None), L.SH(2, 0, None, None), L.SH(0, 2, None, None), L.SH(-1, 0, None, None)):
        assert lib.gs_sh_features(4, ctypes.byref(g), ctypes.byref(bad), fake, 1, fake, fake, None) == \
            L.GS_ERR_INVALID_ARG
    # the constant-band gradient is a sum over views: no views is an error, missing outputs too
    assert lib.gs_sh_features_bwd(4, ctypes.byref(g), ctypes.byref(ok), fake, 0, *([fake] * 8), None) == \
        L.GS_ERR_INVALID_ARG
    assert lib.gs_sh_features_bwd(4, ctypes.byref(g), ctypes.byref(ok), fake, 2, fake, fake, fake, fake, fake, fake,
                                  None, fake, None) == L.GS_ERR_INVALID_ARG


def _learned_bwd_call(drop=None):
    """gs_render_bwd in learned mode with placeholder pointers (never dereferenced on the
    host); `drop` names one argument to leave out."""
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    c.n_sem = 16
    fake = ctypes.c_void_p(256)
    g = L.Gaussians(10, fake, fake, fake, fake, fake, None, fake)
    p = L.Projected(fake, fake, fake)
    h = L.Head()
    h.d_in, h.d_hidden, h.n_classes = 16, 64, 52
    h.W1 = h.b1 = h.W2 = h.b2 = 256
    fwd = L.Images(fake, fake, fake, None, 100, None, 0)
    gin = L.Images(fake, None, None, fake, 100, None, 0)
    gr = L.Grads(*([fake] * 12))
    ws = 1 << 30
    items = fake
    if drop == "emb_grad":
        gr.emb = None
    elif drop == "head_W2_grad":
        gr.head_W2 = None
    elif drop == "logit_grad":
        gin.logits = None
    elif drop == "items":
        items = None
    elif drop == "head":
        h = None
    elif drop == "n_classes":
        h.n_classes = 65
    elif drop == "n_sem":
        c.n_sem = 20
    elif drop == "workspace":
        ws = 16
    return lib.gs_render_bwd(ctypes.byref(c), ctypes.byref(g), ctypes.byref(p), fake, 1, items, 1, 4, fake, fake,
                             ctypes.byref(h) if h is not None else None, ctypes.byref(fwd), ctypes.byref(gin),
                             ctypes.byref(gr), fake, ws, None)


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host-only check: placeholder pointers must never reach a GPU")
def test_invalid_learned_backward_enqueues_nothing():
    """Without a GPU, any launch fails with GS_ERR_HIP. An invalid learned-mode call must come
    back with its argument error instead: nothing was enqueued before the check (the zeroing
    of the outputs included). The complete call is the control: it reaches a launch."""
    for drop in ("emb_grad", "head_W2_grad", "logit_grad", "items", "head", "n_classes", "n_sem"):
        assert _learned_bwd_call(drop) == L.GS_ERR_INVALID_ARG, drop
    assert _learned_bwd_call("workspace") == L.GS_ERR_WORKSPACE
    assert _learned_bwd_call() == L.GS_ERR_HIP


def test_static_loss_refuses_more_items_than_its_scratch_holds():
    """gs_pyramid_loss_static returns GS_ERR_WORKSPACE for more than 2048 items before any
    launch (placeholder pointers, never dereferenced)."""
    lib = L.lib()
    c = L.Config()
    lib.gs_config_default(ctypes.byref(c))
    c.n_sem = 4
    fake = ctypes.c_void_p(256)
    img = L.Images(fake, None, None, None, 100, None, 0)
    t = L.Targets(fake, fake, fake)
    w = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    call = lambda n_items: lib.gs_pyramid_loss_static(  # noqa: E731
        ctypes.byref(c), fake, n_items, 100, 4, ctypes.byref(img), ctypes.byref(t), None, w, fake,
        ctypes.byref(img), None, None)
    assert call(2049) == L.GS_ERR_WORKSPACE
    assert call(-1) == L.GS_ERR_INVALID_ARG
    assert call(0) == L.GS_OK


def test_semantic_colour_loss_arguments_are_checked_on_the_host():
    """The semantic colour loss (eq. 12) needs plain mode with 3 composited semantic channels
    and no class count; a weight outside [0, 1] is refused. Every refusal comes before any
    launch (placeholder pointers; the static entry point refuses on the host before it looks
    up its array)."""
    lib = L.lib()
    fake = ctypes.c_void_p(256)
    w = (ctypes.c_float * 3)(1.0, 1.0, 1.0)

    def call(n_sem=3, n_classes=0, lam_s=0.2, logits=None):
        c = L.Config()
        lib.gs_config_default(ctypes.byref(c))
        c.n_sem = n_sem
        c.sem_ssim_lambda = lam_s
        img = L.Images(fake, None, None, logits, 100, None, 0)
        t = L.Targets(fake, fake, None, fake)
        return lib.gs_pyramid_loss_static(ctypes.byref(c), fake, 3000, 100, n_classes, ctypes.byref(img),
                                          ctypes.byref(t), None, w, fake, ctypes.byref(img), None, None)

    assert call(n_sem=4) == L.GS_ERR_INVALID_ARG
    assert call(n_classes=3) == L.GS_ERR_INVALID_ARG
    assert call(logits=fake) == L.GS_ERR_INVALID_ARG
    assert call(lam_s=1.5) == L.GS_ERR_INVALID_ARG
    assert call(lam_s=-0.1) == L.GS_ERR_INVALID_ARG
    assert call() == L.GS_ERR_WORKSPACE          # valid arguments: refused only for its 3000 items


def test_tile_shapes_accepted_and_refused_on_the_host():
    """256-pixel tiles of width 8, 16, 32 or 64 are accepted; other shapes are refused."""
    lib = L.lib()
    V = (L.View * 1)()
    W = (ctypes.c_int32 * 1)(100)
    H = (ctypes.c_int32 * 1)(60)
    K = (ctypes.c_float * 4)(50.0, 50.0, 50.0, 30.0)
    lv = (ctypes.c_int32 * 1)(1)
    for (tw, th), ok in (((16, 16), True), ((32, 8), True), ((8, 32), True), ((64, 4), True), ((32, 16), False),
                         ((4, 64), False), ((12, 12), False)):
        c = L.Config()
        lib.gs_config_default(ctypes.byref(c))
        c.tile_w, c.tile_h = tw, th
        items = (L.Item * 1)()
        npix, ntile = ctypes.c_int64(), ctypes.c_int32()
        r = lib.gs_make_items(ctypes.byref(c), 1, V, W, H, K, lv, items, ctypes.byref(npix), ctypes.byref(ntile))
        assert (r >= 0) == ok, (tw, th, r)   # the item count, or a negative status
        if ok:
            assert ntile.value == -(-100 // tw) * -(-60 // th)
