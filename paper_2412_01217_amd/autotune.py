"""Autotuner for the batched mapping step.

For one workload signature (Gaussian count, channels, items, pixels, tiles) it times
each candidate launch configuration -- render kernel variant (per-lane FMA, single-precision
or split-bfloat16 matrix cores), tile launch order (coarse pyramid levels first, or item order),
the forward's work item (segments of long lists, or whole lists), the segment length (256,
1024 (the default) or 4096 list entries: the reverse pass's work item and the forward's state
points) and
the screen tile's shape (256 pixels as 16x16, 32x8, 8x32 or 64x4) -- as HIP graph replays of the whole
step, keeps the fastest, then times that configuration with each bin-sort method (radix
passes, or buckets with per-tile sorts in LDS, gs_config.sort_mode 1 and 2) and keeps the
faster, and caches the choice in a JSON file (GS_AUTOTUNE_CACHE, default
~/.cache/gs_autotune.json) keyed by device and signature. Every candidate computes the same
result; only the schedule (and, with the tile shape, the binning) differs. A candidate with
another tile shape needs the item table of that shape: make_step builds its step on
frame_for(cfg, frame).
"""
from __future__ import annotations

import json
import os

import torch

def _c(variant, tile_order, fwd_chunk, tile_w=16, tile_h=16, seg_len=0):
    return {"variant": variant, "tile_order": tile_order, "fwd_chunk": fwd_chunk, "tile_w": tile_w, "tile_h": tile_h,
            "seg_len": seg_len, "sort_mode": 0}


# gs_config.sort_mode 2 (buckets) handles frames of up to this many tiles
BUCKET_MAX_TILES = 12288


# every candidate sets every key, so that none inherits a value from the previous one
CANDIDATES = (_c(3, 0, 0), _c(3, 0, 1), _c(3, 0, 1, seg_len=256), _c(3, 0, 0, seg_len=256),
              _c(3, 0, 0, seg_len=4096), _c(3, 1, 0), _c(2, 0, 1), _c(1, 1, 1),
              _c(3, 0, 1, 32, 8), _c(3, 0, 0, 32, 8), _c(3, 0, 0, 8, 32), _c(3, 0, 0, 64, 4))


def frame_for(cfg, frame):
    """The item table of `frame`'s views for cfg's tile shape (frame itself when the shape
    is the same; built once per shape and kept on frame)."""
    tile = (int(cfg.tile_w), int(cfg.tile_h))
    if tile == frame.tile:
        return frame
    cache = frame.__dict__.setdefault("_tile_frames", {})
    if tile not in cache:
        from . import raster
        cache[tile] = raster.Frame(cfg, frame.views, device=frame.device)
    return cache[tile]


def cache_path() -> str:
    return os.environ.get("GS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gs_autotune.json"))


def signature(cfg, frame, n: int) -> str:
    dev = torch.cuda.get_device_properties(frame.device)
    arch = getattr(dev, "gcnArchName", dev.name).split(":")[0]
    return f"{arch}|n={n}|sem={cfg.n_sem}|items={frame.n_items}|px={frame.n_pixels}|tiles={frame.n_tiles}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass   # a read-only home only costs re-tuning next time


def time_step(step, reps=5, warmup=2) -> float:
    """Mean milliseconds of a graph replay of step.run()."""
    graph = step.capture()
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        graph.launch()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def tune(make_step, cfg, frame, n: int, candidates=CANDIDATES, reps=5, use_cache=True) -> dict:
    """make_step(cfg) -> an object with run() and capture(). Returns
    {"choice": {...}, "times_ms": {...}, "cached": bool}; sets the choice on cfg."""
    key = signature(cfg, frame, n)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        choice = db[key]["choice"]
        for k, v in choice.items():
            setattr(cfg, k, v)
        return {"choice": choice, "times_ms": db[key]["times_ms"], "cached": True}
    times = {}
    best, best_t = None, float("inf")
    for cand in candidates:
        for k, v in cand.items():
            setattr(cfg, k, v)
        step = make_step(cfg)
        t = time_step(step, reps=reps)
        name = ",".join(f"{k}={v}" for k, v in cand.items())
        times[name] = t
        if t < best_t:
            best, best_t = cand, t
        del step
    for k, v in best.items():
        setattr(cfg, k, v)
    if frame_for(cfg, frame).n_tiles <= BUCKET_MAX_TILES:
        base = ",".join(f"{k}={v}" for k, v in best.items() if k != "sort_mode")
        best_t = float("inf")
        pick = dict(best)
        for mode in (1, 2):
            cfg.sort_mode = mode
            step = make_step(cfg)
            t = time_step(step, reps=reps)
            times[f"{base},sort_mode={mode}"] = t
            if t < best_t:
                best_t, pick = t, dict(best, sort_mode=mode)
            del step
        best = pick
        cfg.sort_mode = best["sort_mode"]
    db[key] = {"choice": best, "times_ms": times}
    if use_cache:
        _store(db)
    return {"choice": best, "times_ms": times, "cached": False}
