"""Throughput of the pyramid Gaussian-splatting rasterizer, forward + backward.

One step = projection -> binning/sort -> compositing -> pyramid loss -> backward to
every Gaussian parameter and the pose tangent, over every pyramid level of the
batch, through the C ABI, captured once as a HIP graph and replayed. Inputs are
resident in HBM before timing; targets (2x2 box pyramids of a render of a perturbed
copy of the scene) are built once beforehand.

Prints one JSON line. `value` is the default workload's MP/s: the large two-room scene
(2M Gaussians, 52 classes through the learned 16 -> 64 -> 52 head, its decode fused into
the loss), 16 views at 1920x1080 with 4 pyramid levels each, in the launch configuration
the autotuner picks, with the head first trained on the GPU. The same line carries the
room (200k, plain 52 classes), the 8-view batch (autotuned), learned against plain on the
batch scene and on the large scene, and the room step's variants, unless --quick.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd megapixels/s over all pyramid levels; HBM GB/s; plain vs learned-sem"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak from unit counts: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s,
# doubled by packed-FP32 issue (157.3); the library is built without packed FP32
VALU_PEAK_TFLOPS = 157.3
VALU_PEAK_UNPACKED_TFLOPS = 78.6


# ----------------------------------------------------------------------------- workloads
def make_targets(cfg_plain, fr, sc, device, sem_color=False):
    """rgb, depth, labels: a perturbed copy of the scene rendered at every item, level 0
    box-downsampled to the coarser levels, labels = argmax of the class channels; with
    sem_color (a scene whose semantic feature is a 3-channel colour) the semantic colour
    image instead of labels."""
    import torch
    from paper_2412_01217_amd import raster, scenes
    C = cfg_plain.n_sem
    tgt = scenes.perturbed(sc)
    tgt.emb = None
    gt = raster.to_device(tgt, device)
    pt = raster.preprocess(cfg_plain, gt, fr)
    st = raster.bin_sort(cfg_plain, pt, fr, sc.n)
    timg = raster.render_fwd(cfg_plain, gt, pt, fr, st)
    K = 4 + C
    labels = torch.empty(fr.n_pixels, dtype=torch.int32, device=device)
    raster.downsample(fr, K, timg["color"], labels)
    rgb = torch.empty(3 * fr.n_pixels, dtype=torch.float32, device=device)
    depth = torch.empty(fr.n_pixels, dtype=torch.float32, device=device)
    for it in fr.item_list():
        HW = it["W"] * it["H"]
        pb = it["pixel_base"]
        planes = timg["color"][pb * K: pb * K + K * HW].view(K, HW)
        rgb[pb * 3: pb * 3 + 3 * HW] = planes[:3].reshape(-1)
        depth[pb: pb + HW] = planes[3]
    if sem_color:
        semc = torch.empty(3 * fr.n_pixels, dtype=torch.float32, device=device)
        for it in fr.item_list():
            HW = it["W"] * it["H"]
            pb = it["pixel_base"]
            semc[pb * 3: pb * 3 + 3 * HW] = timg["color"][pb * K: pb * K + K * HW].view(K, HW)[4:7].reshape(-1)
        torch.cuda.synchronize()
        return dict(rgb=rgb, depth=depth, sem_color=semc)
    torch.cuda.synchronize()
    return dict(rgb=rgb, depth=depth, label=labels)


def plain_step(sc, views, device, targets=None, variant=0, tile_order=0, ssim_lambda=0.0, isotropic=0, sh=None,
               sem_ssim_lambda=None):
    """sh: (rgb degree, semantic degree) of seeded SH bands N(0, 0.1), or None.
    sem_ssim_lambda: not None for a scene whose semantic feature is a 3-channel colour,
    trained with eq. 12's loss at that lambda_s against a semantic colour target."""
    import torch
    from paper_2412_01217_amd import raster
    from paper_2412_01217_amd.step import MappingStep
    C = sc.n_classes
    cfg = raster.config(C, variant=variant, tile_order=tile_order, ssim_lambda=float(ssim_lambda),
                        isotropic=int(isotropic), view_features=int(sh is not None),
                        sem_ssim_lambda=float(sem_ssim_lambda or 0.0))
    fr = raster.Frame(cfg, views, device=device)
    g = raster.to_device(sc, device)
    g.pop("emb", None)
    semc = sem_ssim_lambda is not None
    targets = targets if targets is not None else make_targets(cfg, fr, sc, device, sem_color=semc)
    if semc:
        return MappingStep(cfg, fr, g, targets, 0), targets
    shd = None
    if sh is not None:
        rng = np.random.default_rng(7000)
        dr, ds = sh
        band = lambda d, ch: (torch.tensor(rng.normal(size=(sc.n, (d + 1) ** 2 - 1, ch)) * 0.1,  # noqa: E731
                                           dtype=torch.float32, device=device) if d else None)
        shd = dict(rgb_degree=dr, sem_degree=ds, rgb_rest=band(dr, 3), sem_rest=band(ds, C))
    return MappingStep(cfg, fr, g, targets, C, sh=shd), targets


def learned_step(sc, views, head, device, targets, cfg=None):
    """The learned mapping step (decode, cross-entropy and the decode's backward inside the
    loss call)."""
    from paper_2412_01217_amd import raster
    from paper_2412_01217_amd.step import MappingStep
    cfg = cfg or raster.config(16)
    fr = raster.Frame(cfg, views, device=device)
    g = raster.to_device(sc, device)
    g.pop("sem", None)
    return MappingStep(cfg, fr, g, targets, head["b2"].shape[0], head=head)


def train_head(sc, device, steps, heldout_views, seed_offset):
    """Fits the embedding and the 16 -> 64 -> C head to the plain C-class render on the GPU
    (a fresh random 640x480 view with 3 levels per step), then measures argmax agreement
    and logit error on held-out views. Returns (report, head dict, scene copy with the
    trained embedding)."""
    import torch
    from paper_2412_01217_amd import scenes
    from paper_2412_01217_amd.learned import Trainer

    def train_views(k):
        return scenes.room_views(sc, 1, 640, 480, levels=3, seed=scenes.SEED_VIEWS + seed_offset + k)[0]
    t0 = time.perf_counter()
    tr = Trainer(sc, train_views, sc.n_classes, device)
    before = tr.evaluate(heldout_views[:1])
    tr.train(steps)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    quality = tr.evaluate(heldout_views)
    head = tr.head.as_dict()
    trained = sc.copy()
    trained.emb = tr.g_learned["emb"].cpu().numpy().view(np.uint16).copy()
    del tr
    torch.cuda.empty_cache()
    rep = {"head_training": {"steps": steps, "seconds": train_s, "train_views": "a fresh random 640x480 view "
                             "(3 levels) per step", "agreement_untrained": before["agreement"]},
           "argmax_agreement": quality["agreement"], "logit_rmse": quality["logit_rmse"],
           "heldout_views": len(heldout_views), "heldout_pixels": quality["pixels"]}
    return rep, head, trained


# ----------------------------------------------------------------------------- measurement
def measure(step, steps, warmup, graph=True):
    """Per-stage times from an eager pass with events between the calls, then the timed
    region: `steps` graph replays of the whole step."""
    import torch
    from paper_2412_01217_amd import raster
    for _ in range(warmup):
        step.run()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(steps):
        step.run(evs[k])
    t1.record()
    torch.cuda.synchronize()
    eager_ms = t0.elapsed_time(t1) / steps
    names = ("bin_sort", "render_fwd", "loss", "render_bwd")
    stage_ms = {nm: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, nm in enumerate(names)}
    stage_ms["preprocess_and_gaps"] = eager_ms - sum(stage_ms.values())
    run = step.run
    if graph:
        g = raster.Graph(step.run, step.frame.device)
        run = g.launch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        run()
    t1.record()
    torch.cuda.synchronize()
    assert not step.overflowed()
    ms = t0.elapsed_time(t1) / steps
    # the spread of single replays, from a second set of `steps` replays with an event
    # between every two (outside the timed region above)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    marks[0].record()
    for k in range(steps):
        run()
        marks[k + 1].record()
    torch.cuda.synchronize()
    per = np.array([marks[k].elapsed_time(marks[k + 1]) for k in range(steps)])
    spread = {"median": float(np.median(per)), "p90": float(np.percentile(per, 90)), "replays": steps}
    return dict(ms=ms, eager_ms=eager_ms, stage_ms=stage_ms, step_ms_spread=spread)


def gpu_clocks():
    """The clock lines of `rocm-smi --showclocks` (a read-only query run as a child
    process), or None."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=30)
    except (OSError, subprocess.SubprocessError):
        return None
    lines = [ln.strip() for ln in r.stdout.splitlines() if "clk" in ln and ":" in ln]
    return lines or None


def host_cpu():
    """Model name and logical CPU count of the host that runs the CPU baseline."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def work_counts(step):
    import torch
    fr = step.frame
    nc = int(step.img["n_contrib"].to(torch.int64).sum().item())
    return dict(pairs=nc, dup=step.n_dup_probe, visible=step.n_visible_probe, pixels=fr.n_pixels, items=fr.n_items,
                views=fr.n_views, n=step.n, K=4 + step.cfg.n_sem)


def algorithmic_bytes(c, n_classes, learned=False):
    """Bytes the step must move at minimum (model documented with the design notes)."""
    N, V, E, vis, D, P, K = c["n"], c["views"], c["items"] * c["n"], c["visible"], c["dup"], c["pixels"], c["K"]
    feat = 4 * (K - 1) if not learned else 12 + 32            # rgb + semantics (float) or embedding (bf16)
    rec = 32 + 4                                               # render record + depth
    tile_passes = 2
    b = 0
    b += V * N * 44 + E * 4 + vis * 36                          # projection
    b += E * 4 + vis * 12 * (1 + 2 * 5) + D * 8 * (1 + 2 * tile_passes) + D * 8   # binning and sort
    b += D * (4 + rec + feat) + P * 4 * (K + 2)                # forward
    if learned:
        b += P * 4 * (16 + n_classes)                          # decode: embedding in, logits out
    b += P * 4 * (K + 5) + P * 4 * K                           # loss
    b += D * (4 + rec + feat) + P * 4 * (K + 2) + D * 4 * (K + 6)   # backward compositing
    b += V * N * 44 + vis * 32 + N * (44 + 4 * (K - 1))        # projection backward + gradient writes
    return b


# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries per workload (the render kernels'
# HBM bytes per launch, with the source hash they were taken on)
COUNTERS = {"room": os.path.join(ROOT, "profiles", "render_room200k_c52_hbm_counters.md"),
            "large": os.path.join(ROOT, "profiles", "render_large2m_c52_learned_hbm_counters.md")}


def measured_traffic(workload):
    """HBM bytes per launch of the render kernels on `workload`, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (scaled by the copy calibration there), or {}
    when the render source has changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(COUNTERS[workload]).read()
        src = open(os.path.join(ROOT, "paper_2412_01217_amd", "csrc", "render_split.hip"), "rb").read()
    except (OSError, KeyError):
        return {}
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != hashlib.sha256(src).hexdigest():
        return {}
    return {k: float(v) for k, v in re.findall(r"traffic (k_render_\w+): ([0-9.e+]+) bytes", text)}


def roofline(step, stage_ms, counts, traffic=None):
    K = counts["K"]
    nc = counts["pairs"]
    traffic = traffic or {}
    kern = {}
    for name, stage, per_pair in (("k_render_fwd", "render_fwd", 18 + 2 * K), ("k_render_bwd", "render_bwd", 45 + 6 * K)):
        flops = nc * per_pair
        t = stage_ms[stage]
        ach = flops / (t * 1e-3) / 1e12
        kern[name] = {"bound": "alu", "kernel": name, "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": ach / VALU_PEAK_TFLOPS, "frac_unpacked_peak": ach / VALU_PEAK_UNPACKED_TFLOPS,
                      "traffic": traffic.get(name), "flops_per_launch": flops, "avg_launch_ms": t,
                      "timed_call": "gs_" + stage}
    dominant = max(kern, key=lambda k: kern[k]["avg_launch_ms"])
    return kern[dominant], {k: v for k, v in kern.items() if k != dominant}


# ----------------------------------------------------------------------------- sub-benchmarks
def batch_report(args, device):
    """The 8-view batch (500k Gaussians, 20 classes, 640x480, 1-3 levels each), with the
    launch configuration picked by the autotuner."""
    from paper_2412_01217_amd import autotune, scenes
    from paper_2412_01217_amd.step import MappingStep
    sc, views = scenes.config_batch()
    step, targets = plain_step(sc, views, device)

    def make(cfg):
        return MappingStep(cfg, autotune.frame_for(cfg, step.frame), step.g, targets, sc.n_classes)

    tuned = autotune.tune(make, step.cfg, step.frame, sc.n)
    step = make(step.cfg)
    m = measure(step, args.steps, args.warmup)
    c = work_counts(step)
    return {"workload": "room 6x5x3 m, 500k Gaussians, 20 plain classes, 8 views 640x480, 1-3 levels each",
            "value": c["pixels"] / 1e6 / (m["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": m["ms"],
            "stage_ms": m["stage_ms"], "items": c["items"], "pixels_per_step": c["pixels"], "duplicates": c["dup"],
            "autotune": tuned,
            "hbm_gbs_effective": algorithmic_bytes(c, sc.n_classes) / (m["ms"] * 1e-3) / 1e9}


def learned_report(args, device):
    """The learned semantic head on the batched room scene with 52 classes: train the
    head for --train-steps steps on plain renders of random views, measure argmax agreement
    and logit error on 16 held-out views, then time learned against plain on the 8-view batch."""
    import torch
    from paper_2412_01217_amd import scenes
    sc, views = scenes.config_learned()
    test_views = scenes.room_views(sc, 16, 640, 480, levels=3, seed=scenes.SEED_VIEWS + 61)
    rep, head, trained_sc = train_head(sc, device, args.train_steps, test_views, 10000)
    plain, targets = plain_step(sc, views, device)
    mp = measure(plain, args.steps, args.warmup)
    cp = work_counts(plain)
    del plain
    torch.cuda.empty_cache()
    lstep = learned_step(trained_sc, views, head, device, targets)
    ml = measure(lstep, args.steps, args.warmup)
    cl = work_counts(lstep)
    mpx = cl["pixels"] / 1e6
    return {"workload": "room 6x5x3 m, 500k Gaussians, 52 classes via 16-dim bf16 embedding + 16->64->52 MLP, "
                        "8 views 640x480, 1-3 levels each", **rep,
            "learned": {"value": mpx / (ml["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": ml["ms"],
                        "stage_ms": ml["stage_ms"],
                        "hbm_gbs_effective": algorithmic_bytes(cl, 52, learned=True) / (ml["ms"] * 1e-3) / 1e9},
            "plain_c52": {"value": mpx / (mp["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": mp["ms"],
                          "stage_ms": mp["stage_ms"],
                          "hbm_gbs_effective": algorithmic_bytes(cp, 52) / (mp["ms"] * 1e-3) / 1e9},
            "speedup_learned_over_plain": mp["ms"] / ml["ms"]}


# candidates timed for the large workload (the per-lane FMA variant, several times slower on
# every workload measured, is left out to keep the tuning short)
def large_candidates():
    from paper_2412_01217_amd import autotune
    return [c for c in autotune.CANDIDATES if c["variant"] != 1]


def large_headline(args, dev):
    """The large workload: two rooms, 2M Gaussians, 52 classes through the learned head,
    16 views at 1920x1080 with 4 levels. Trains the head (640x480 views of this scene),
    autotunes the launch configuration, then times the learned step."""
    import torch
    from paper_2412_01217_amd import autotune, raster, scenes
    sc, views = scenes.config_large()
    cfg_p = raster.config(52)
    fr_p = raster.Frame(cfg_p, views, device=dev)
    targets = make_targets(cfg_p, fr_p, sc, dev)
    torch.cuda.empty_cache()
    heldout = scenes.room_views(sc, 2, 1920, 1080, levels=4, seed=scenes.SEED_VIEWS + 64)
    rep, head, trained_sc = train_head(sc, dev, args.train_steps, heldout, 40000)
    cfg = raster.config(16)
    step = learned_step(trained_sc, views, head, dev, targets, cfg=cfg)

    def make(c):
        from paper_2412_01217_amd.step import MappingStep
        return MappingStep(c, autotune.frame_for(c, step.frame), step.g, targets, 52, head=head)
    tuned = autotune.tune(make, cfg, step.frame, sc.n, candidates=large_candidates(), reps=3)
    step = make(cfg)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    c = work_counts(step)
    return sc, views, targets, head, trained_sc, step, m, c, tuned, rep


def large_plain_report(args, dev, sc, views, targets, ms_learned):
    """The plain 52-class render of the large workload (logits composited per Gaussian) in
    the autotuner's configuration, beside the learned form."""
    import torch
    from paper_2412_01217_amd import autotune
    from paper_2412_01217_amd.step import MappingStep
    step, _ = plain_step(sc, views, dev, targets=targets)

    def make(c):
        return MappingStep(c, autotune.frame_for(c, step.frame), step.g, targets, 52)
    tuned = autotune.tune(make, step.cfg, step.frame, sc.n, candidates=large_candidates(), reps=2)
    step = make(step.cfg)
    m = measure(step, max(3, args.steps // 4), 2, graph=not args.eager)
    px = step.frame.n_pixels
    del step
    torch.cuda.empty_cache()
    return {"workload": "the large workload with the plain 52-class render", "value": px / 1e6 / (m["ms"] * 1e-3),
            "unit": "MP/s", "ms_per_step": m["ms"], "stage_ms": m["stage_ms"], "autotune": tuned,
            "speedup_learned_over_plain": m["ms"] / ms_learned}


def cpu_baseline(sc, views, targets, C, min_s=10.0):
    """The FP64 oracle (single thread) on the whole room workload: forward + loss + backward
    over every pixel of every pyramid level (7-15 s of one core per run), repeated until at
    least min_s seconds have been timed."""
    import oracle
    n_items, P, tiles = oracle.layout(views)
    tgt = {k: v.cpu().numpy() for k, v in targets.items()}
    total, reps = 0.0, 0
    while total < min_s:
        t0 = time.perf_counter()
        r = oracle.render(oracle.Config(), sc, views)
        _, gimg = oracle.loss(views, C, r["img"], tgt["rgb"], tgt["depth"], tgt["label"])
        oracle.backward(oracle.Config(), sc, views, gimg)
        total += time.perf_counter() - t0
        reps += 1
    return dict(value=P * reps / total / 1e6, unit="MP/s", cores=1, kind="oracle",
                sample=f"the whole workload ({n_items} levels, {tiles} tiles, {P} px), forward + loss + backward "
                       f"including the projection and binning of all {sc.n} Gaussians; {reps} runs, {total:.1f} s")


def cpu_baseline_large(sc, views, targets, head, stride=4):
    """The FP64 oracle (single thread) on a sample of the large learned workload: view 0 with
    its 4 levels, every `stride`-th tile of each level; forward (projection and binning of
    all Gaussians included), the head's decode, the loss, the head's backward and the render
    backward, once. MP/s counts the sampled tiles' pixels."""
    import oracle
    from paper_2412_01217_amd import scenes
    v0 = views[:1]
    its = oracle.items(v0)
    n_items, P0, tiles = oracle.layout(v0)
    mask = (np.arange(tiles) % stride == 0).astype(np.uint8)
    sel = np.zeros(P0, bool)
    for it in its:
        vv, uu = np.mgrid[0:it["H"], 0:it["W"]]
        t = it["tile0"] + (vv // 16) * it["ntx"] + (uu // 16)
        sel[it["pix0"]: it["pix0"] + it["W"] * it["H"]] = mask[t.reshape(-1)] != 0
    C = int(head["b2"].shape[0])
    w = {k: (scenes.bf16_bits_to_f32(head[k].cpu().numpy().view(np.uint16)) if k in ("W1", "W2")
             else head[k].cpu().numpy()).astype(np.float64) for k in ("W1", "b1", "W2", "b2")}
    emb = scenes.bf16_bits_to_f32(sc.emb).astype(np.float64)
    t_rgb = targets["rgb"][:3 * P0].cpu().numpy()
    t_depth = targets["depth"][:P0].cpu().numpy()
    t_lab = np.where(sel, targets["label"][:P0].cpu().numpy(), -1).astype(np.int32)
    cfg = oracle.Config()
    t0 = time.perf_counter()
    r = oracle.render(cfg, sc, v0, sem=emb, tile_mask=mask)
    K = 20
    E = np.concatenate([r["img"][it["pix0"] * K: it["pix0"] * K + K * it["W"] * it["H"]].reshape(K, -1).T[:, 4:]
                        for it in its])
    logits = np.zeros((P0, C))
    logits[sel] = oracle.head_forward(E[sel], w["W1"], w["b1"], w["W2"], w["b2"])
    img_l = np.zeros(P0 * (4 + C))
    for it in its:
        HW = it["W"] * it["H"]
        src = r["img"][it["pix0"] * K: it["pix0"] * K + K * HW].reshape(K, HW)
        dst = img_l[it["pix0"] * (4 + C): it["pix0"] * (4 + C) + (4 + C) * HW].reshape(4 + C, HW)
        dst[:4] = src[:4]
        dst[4:] = logits[it["pix0"]: it["pix0"] + HW].T
    _, g_l = oracle.loss(v0, C, img_l, t_rgb, t_depth, t_lab)
    glog = np.concatenate([g_l[it["pix0"] * (4 + C): it["pix0"] * (4 + C) + (4 + C) * it["W"] * it["H"]]
                           .reshape(4 + C, -1).T[:, 4:] for it in its])
    hb = oracle.head_backward(E[sel], w["W1"], w["b1"], w["W2"], glog[sel])
    gimg = np.zeros(P0 * K)
    dE = np.zeros((P0, 16))
    dE[sel] = hb["E"]
    for it in its:
        HW = it["W"] * it["H"]
        src = g_l[it["pix0"] * (4 + C): it["pix0"] * (4 + C) + (4 + C) * HW].reshape(4 + C, HW)
        dst = gimg[it["pix0"] * K: it["pix0"] * K + K * HW].reshape(K, HW)
        dst[:4] = src[:4] * sel[it["pix0"]: it["pix0"] + HW]
        dst[4:] = dE[it["pix0"]: it["pix0"] + HW].T
    oracle.backward(cfg, sc, v0, gimg, sem=emb, tile_mask=mask)
    total = time.perf_counter() - t0
    n_px = int(sel.sum())
    return dict(value=n_px / total / 1e6, unit="MP/s", cores=1, kind="oracle",
                sample=f"view 0 of the large workload (its {n_items} levels), every {stride}th tile: {n_px} of "
                       f"{P0} px; forward (projection and binning of all {sc.n} Gaussians per level), decode, loss, "
                       f"head backward and render backward; {total:.1f} s")


def adam_report(step, steps):
    """The mapping update after the step's backward: one Adam launch over every Gaussian
    parameter group (HBM-bound: 4 float reads and 3 writes per element), timed on the
    step's own gradients."""
    import torch
    from paper_2412_01217_amd import raster
    g = step.g
    m = {k: torch.zeros_like(t) for k, t in g.items() if k in raster.PARAM_FIELDS and t is not None}
    v = {k: torch.zeros_like(t) for k, t in g.items() if k in raster.PARAM_FIELDS and t is not None}
    saved = {k: t.clone() for k, t in m.items()}
    saved_g = {k: g[k].clone() for k in m}
    hp = raster.adam_config(dict(mean=1e-6, log_scale=1e-6, quat=1e-6, opacity=1e-6, rgb=1e-6, sem=1e-6))
    for i in range(3):
        raster.gaussians_adam(g, step.grads, m, v, hp, i + 1)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        raster.gaussians_adam(g, step.grads, m, v, hp, i + 4)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    for k in m:                                    # leave the scene as it was
        g[k].copy_(saved_g[k])
    del saved
    elems = sum(t.numel() for t in m.values())
    gbs = 28.0 * elems / (ms * 1e-3) / 1e9
    return {"kernel": "k_adam_groups", "elements": elems, "avg_launch_ms": ms, "algorithmic_bytes": 28 * elems,
            "achieved_gbs": gbs, "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                              "frac": gbs / HBM_PEAK_GBS}}


def isotropic_report(args, dev, sc, views, targets):
    """The room step with the literal primitive of eq. 1-3 (one scale per Gaussian, the
    first of the scene's three, no rotation) in place of the EWA footprint."""
    import torch
    step, _ = plain_step(sc, views, dev, targets=targets, variant=args.variant, isotropic=1)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    c = work_counts(step)
    del step
    torch.cuda.empty_cache()
    return {"primitive": "isotropic (eq. 1-3)", "value": c["pixels"] / 1e6 / (m["ms"] * 1e-3), "unit": "MP/s",
            "ms_per_step": m["ms"], "stage_ms": m["stage_ms"], "duplicates": c["dup"], "pairs_iterated": c["pairs"]}


def sh_report(args, dev, sc, views, targets, degrees=(3, 1)):
    """The room step with view-dependent features: SH of degree 3 for colour and 1 for the
    52 class logits, evaluated per view before the render and differentiated after it."""
    import torch
    step, _ = plain_step(sc, views, dev, targets=targets, variant=args.variant, sh=degrees)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    c = work_counts(step)
    del step
    torch.cuda.empty_cache()
    return {"sh_degrees": {"rgb": degrees[0], "semantics": degrees[1]},
            "value": c["pixels"] / 1e6 / (m["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": m["ms"],
            "stage_ms": m["stage_ms"]}


def semantic_colour_report(args, dev, sc, views, lam=0.2):
    """The room step with the paper's semantic colour feature (3 channels per Gaussian, its
    class's colour) and its full loss: eq. 10 and eq. 12 with lambda_r = lambda_s = 0.2."""
    import torch
    from paper_2412_01217_amd import scenes
    sc3 = scenes.semantic_colour_scene(sc)
    step, _ = plain_step(sc3, views, dev, variant=args.variant, ssim_lambda=lam, sem_ssim_lambda=lam)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    px = step.frame.n_pixels
    del step
    torch.cuda.empty_cache()
    return {"semantic_feature": "3-channel semantic colour", "ssim_lambda": lam, "sem_ssim_lambda": lam,
            "value": px / 1e6 / (m["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": m["ms"], "stage_ms": m["stage_ms"]}


def ssim_report(args, dev, sc, views, targets, ms_ref, loss_ms_ref, lam=0.2):
    """The same room step with the colour loss of eq. 10 at the paper's lambda = 0.2
    (L1 and SSIM) in place of the plain L1 term."""
    import torch
    lam = lam if args.ssim_lambda == 0.0 else 0.0
    step, _ = plain_step(sc, views, dev, targets=targets, variant=args.variant, ssim_lambda=lam)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    px = step.frame.n_pixels
    del step
    torch.cuda.empty_cache()
    return {"ssim_lambda": lam, "value": px / 1e6 / (m["ms"] * 1e-3), "unit": "MP/s", "ms_per_step": m["ms"],
            "loss_stage_ms": m["stage_ms"]["loss"], "compared_to": {"ssim_lambda": args.ssim_lambda,
                                                                      "ms_per_step": ms_ref,
                                                                      "loss_stage_ms": loss_ms_ref}}


# ----------------------------------------------------------------------------- main
def room_headline(args, dev):
    """The room workload (200k Gaussians, 52 plain classes, 1200x680 with 3 levels) in the
    default launch configuration."""
    from paper_2412_01217_amd import scenes
    sc, views = scenes.config_room()
    sh = tuple(int(x) for x in args.sh.split(",")) if args.sh else None
    step, targets = plain_step(sc, views, dev, variant=args.variant, ssim_lambda=args.ssim_lambda, sh=sh)
    m = measure(step, args.steps, args.warmup, graph=not args.eager)
    c = work_counts(step)
    return sc, views, targets, step, m, c, sh


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=("large", "room", "batch", "learned"))
    ap.add_argument("--quick", action="store_true", help="only the timed workload (no sub-reports)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=0, help="room: render kernels 0 auto (3), 1 VALU, 2 FP32 matrix cores, 3 split-bf16 matrix cores")
    ap.add_argument("--eager", action="store_true", help="time eager calls instead of graph replays")
    ap.add_argument("--sh", default="", metavar="R,S",
                    help="room: SH degrees (colour, semantics) of view-dependent features in the timed step")
    ap.add_argument("--ssim-lambda", type=float, default=0.0,
                    help="room: SSIM weight of the colour loss in the timed step (0: the L1 loss of the workloads)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times): the reference for HBM byte counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    # queried before this process initialises the GPU; skipped under --quick, whose runs are
    # the profiled ones (a profiler refuses the query's child process)
    clocks = None if args.quick else gpu_clocks()
    import torch
    dev = "cuda:0"
    torch.cuda.set_device(0)
    sub = {"batch": batch_report, "learned": learned_report}.get(args.workload)
    if sub is not None:
        print(json.dumps({"metric": METRIC, **sub(args, dev)}), flush=True)
        return
    common = {"metric": METRIC, "unit": "MP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload == "large":
        sc, views, targets, head, trained_sc, step, m, c, tuned, quality = large_headline(args, dev)
        ms = m["ms"]
        roof, other = roofline(step, m["stage_ms"], c, measured_traffic("large"))
        out = {**common, "value": c["pixels"] / 1e6 / (ms * 1e-3), "ms_per_step": ms,
               # compositing, loss and gradients in single precision; the channel contractions on
               # bfloat16 matrix cores with hi/lo split operands (about 2^-16 relative), the decode
               # with bfloat16 weights and hi/lo split activations
               "dtype": "f32 (contractions as split-bf16 MFMA)",
               "config": {"workload": "two-room 12x10x3 m, 2M Gaussians, 52 classes via the learned 16->64->52 head "
                                      "(decode fused into the loss), 16 views 1920x1080, 4-level pyramid",
                          "gaussians": sc.n, "classes": 52, "pixels_per_step": c["pixels"], "items": c["items"],
                          "duplicates": c["dup"], "visible_item_gaussians": c["visible"], "pairs_iterated": c["pairs"],
                          "semantic_mode": "learned", "launch": tuned["choice"]},
               "timed": "eager calls" if args.eager else "HIP graph replay of the whole step",
               "eager_ms_per_step": m["eager_ms"], "step_ms_spread": m["step_ms_spread"], "stage_ms": m["stage_ms"],
               "hbm_gbs_effective": algorithmic_bytes(c, 52, learned=True) / (ms * 1e-3) / 1e9,
               "roofline": roof, "roofline_other": other, "autotune": tuned, "learned_head": quality,
               "gpu_clocks_at_start": clocks}
        del step
        torch.cuda.empty_cache()
        if not args.quick:
            out["large_plain_c52"] = large_plain_report(args, dev, sc, views, targets, ms)
            torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_large(trained_sc, views, targets, head)
            out["cpu_baseline"]["host"] = host_cpu()
        del targets, head, trained_sc
        torch.cuda.empty_cache()
        if not args.quick:
            rsc, rviews, rtargets, rstep, rm, rc, _ = room_headline(args, dev)
            rroof, rother = roofline(rstep, rm["stage_ms"], rc, measured_traffic("room") if args.variant == 0 else {})
            out["room"] = {"workload": "room 6x5x3 m, 200k Gaussians, 52 plain classes, 1 view 1200x680, 3-level "
                                       "pyramid", "value": rc["pixels"] / 1e6 / (rm["ms"] * 1e-3), "unit": "MP/s",
                           "ms_per_step": rm["ms"], "step_ms_spread": rm["step_ms_spread"], "stage_ms": rm["stage_ms"],
                           "duplicates": rc["dup"], "pairs_iterated": rc["pairs"],
                           "hbm_gbs_effective": algorithmic_bytes(rc, 52) / (rm["ms"] * 1e-3) / 1e9,
                           "roofline": rroof, "roofline_other": rother}
            out["mapping_update"] = adam_report(rstep, args.steps)
            del rstep
            torch.cuda.empty_cache()
            out["room"]["with_ssim"] = ssim_report(args, dev, rsc, rviews, rtargets, rm["ms"], rm["stage_ms"]["loss"])
            torch.cuda.empty_cache()
            out["room"]["isotropic_primitive"] = isotropic_report(args, dev, rsc, rviews, rtargets)
            torch.cuda.empty_cache()
            out["room"]["sh_features"] = sh_report(args, dev, rsc, rviews, rtargets)
            torch.cuda.empty_cache()
            out["room"]["semantic_colour_eq12"] = semantic_colour_report(args, dev, rsc, rviews)
            torch.cuda.empty_cache()
            out["batch"] = batch_report(args, dev)
            torch.cuda.empty_cache()
            out["learned_vs_plain"] = learned_report(args, dev)
            torch.cuda.empty_cache()
        print(json.dumps(out), flush=True)
        return
    # --workload room
    sc, views, targets, step, m, c, sh = room_headline(args, dev)
    ms = m["ms"]
    roof, other = roofline(step, m["stage_ms"], c, measured_traffic("room") if args.variant == 0 else {})
    out = {**common, "value": c["pixels"] / 1e6 / (ms * 1e-3), "ms_per_step": ms,
           "dtype": "f32 (contractions as split-bf16 MFMA)",
           "config": {"workload": "room 6x5x3 m, 200k Gaussians, 52 plain classes, 1 view 1200x680, 3-level pyramid",
                      "gaussians": sc.n, "classes": sc.n_classes, "pixels_per_step": c["pixels"], "items": c["items"],
                      "duplicates": c["dup"], "visible_item_gaussians": c["visible"], "pairs_iterated": c["pairs"],
                      "semantic_mode": "plain", "render_variant": args.variant, "ssim_lambda": args.ssim_lambda,
                      "sh_degrees": list(sh) if sh else None},
           "timed": "eager calls" if args.eager else "HIP graph replay of the whole step",
           "eager_ms_per_step": m["eager_ms"], "step_ms_spread": m["step_ms_spread"], "stage_ms": m["stage_ms"],
           "hbm_gbs_effective": algorithmic_bytes(c, sc.n_classes) / (ms * 1e-3) / 1e9,
           "roofline": roof, "roofline_other": other, "gpu_clocks_at_start": clocks}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, views, targets, sc.n_classes)
        out["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
