"""Autotuner for the build's tile shape.

For one image shape (H, W, C, bins, dtype, moments, layout) it times every
legal tile shape of ``ih_build`` on the device with HIP events and keeps the
fastest.  Results are cached in a JSON file (``IH_TUNE_CACHE``, default
``tune_cache.json`` next to this module) keyed by the shape and the device
name, so a shape is tuned once per device.
"""
from __future__ import annotations

import itertools
import json
import os
import threading
from typing import Dict, List, Optional, Tuple

import torch

from . import ih

_CACHE_PATH = os.environ.get("IH_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                          "tune_cache.json"))
_lock = threading.Lock()
_cache: Optional[Dict[str, List[int]]] = None


def _load() -> Dict[str, List[int]]:
    global _cache
    if _cache is None:
        try:
            with open(_CACHE_PATH) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def _save():
    tmp = _CACHE_PATH + ".tmp%d" % os.getpid()
    try:
        with open(tmp, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)
        os.replace(tmp, _CACHE_PATH)
    except OSError:
        pass


def key(H, W, C, bins, dtype, moments, layout, device=None) -> str:
    name = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "cpu"
    return "%s|%dx%dx%d|b%d|%s|m%d|%s" % (name, C, H, W, bins, str(dtype).replace("torch.", ""),
                                          int(bool(moments)), layout)


def candidates(H, W, C, bins, moments, layout) -> List[ih.TileCfg]:
    """Every tile shape the library accepts for this image (filtered by size)."""
    out = []
    if layout == "bhw":
        for th, tw, pg in itertools.product((8, 16, 32, 64, 128), (64, 128, 256), (1, 2, 4, 8, 16)):
            if th * tw > 32768 or (moments and pg * tw // 64 > 32) or pg > max(1, 2 * bins):
                continue
            if th > 2 * H or tw > 2 * max(W, 64):
                continue
            out.append(ih.TileCfg(th, tw, pg))
    else:
        for th, tw in itertools.product((4, 8, 16, 32, 64, 128), (16, 32, 64)):
            if moments and tw > 32:
                continue
            if th > 2 * H or tw > 2 * max(W, 16):
                continue
            out.append(ih.TileCfg(th, tw, 64))
    return out


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(img: torch.Tensor, bins: int, value_bits: Optional[int] = None, moments: bool = False,
         layout: str = "bhw", reps: int = 5, force: bool = False, verbose: bool = False
         ) -> Tuple[ih.TileCfg, Dict[str, float]]:
    """Return the fastest tile shape for this image shape (cached per device)."""
    if img.dim() == 2:
        img = img.unsqueeze(0)
    C, H, W = img.shape
    k = key(H, W, C, bins, img.dtype, moments, layout, img.device)
    with _lock:
        cache = _load()
        if not force and k in cache:
            return ih.TileCfg(*cache[k]), {}
    P = C * bins
    shp = ih.shape_of(P, H, W, layout)
    out = torch.empty(shp, dtype=torch.int32, device=img.device)
    mom = (torch.empty_like(out), torch.empty_like(out)) if moments else None
    cands = candidates(H, W, C, bins, moments, layout)
    ws_need = max(ih.workspace_size(H, W, C, bins, moments, c, layout) for c in cands)
    ws = torch.empty(ws_need, dtype=torch.uint8, device=img.device)
    times: Dict[str, float] = {}
    best, best_t = None, float("inf")
    for cfg in cands:
        t = _time(lambda: ih.ih_build(img, bins, value_bits, moments, cfg, out, mom, ws, layout), reps)
        times[repr(cfg)] = t
        if verbose:
            print("tune %s %s: %.4f ms" % (k, cfg, t), flush=True)
        if t < best_t:
            best, best_t = cfg, t
    with _lock:
        cache = _load()
        cache[k] = list(best.key())
        _save()
    return best, times


def batch_candidates(layout: str) -> List[ih.TileCfg]:
    """Uniform tile shapes tried for a whole batch (every frame gets the same one)."""
    if layout == "hwb":
        return [ih.TileCfg(th, tw, 64) for th, tw in itertools.product((32, 64, 128), (16, 32, 64))]
    return [ih.TileCfg(th, tw, pg) for th, tw, pg in itertools.product((32, 64, 128), (64, 128, 256), (1, 2))
            if th * tw <= 32768]


def tune_batch(frames, metric: str = "chi2", layout: str = "bhw", reps: int = 3,
               verbose: bool = False) -> Tuple[ih.TileCfg, Dict[str, float]]:
    """Tile shape for a batch, chosen by timing the whole batch (all phases, one
    launch per phase) with each candidate shape applied to every frame.  In a
    batch the parallelism comes from many frames at once, so the best shape
    differs from the best shape of each frame built alone.  Frames are dicts as
    for ih.Batch; their own "tile" entries are ignored."""
    times: Dict[str, float] = {}
    best, best_t = None, float("inf")
    for cfg in batch_candidates(layout):
        if layout == "bhw" and any(cfg.planes_per_wave > max(1, int(f["bins"])) for f in frames):
            continue
        fr = [dict(f, tile=cfg, layout=layout) for f in frames]
        try:
            b = ih.Batch(fr, metric, layout=layout)
        except ih.IHError:
            continue
        t = _time(lambda: b.run("phased"), reps)
        del b
        times[repr(cfg)] = t
        if verbose:
            print("tune batch %s: %.4f ms" % (cfg, t), flush=True)
        if t < best_t:
            best, best_t = cfg, t
    if best is None:
        raise ih.IHError("no tile shape fits every frame of the batch")
    return best, times


def tune_batch_classes(frames, metric: str = "chi2", layout: str = "bhw", reps: int = 3, rounds: int = 1,
                       verbose: bool = False):
    """A tile shape per class of frames (the frames with the same bin count),
    chosen by timing the whole batch: start from the best shape for every
    frame (tune_batch), then for each class in turn try every candidate shape
    on its frames while the other classes keep theirs, keeping a change only
    when the whole batch gets faster; `rounds` passes over the classes.  With
    layout="any" a class's candidates are the shapes of both layouts, so each
    class also gets its layout (frames whose planes fill few lanes of a
    planes-innermost wave may build faster bin-major, and the reverse).
    Returns (a (layout, tile) per frame, {bins: (layout, tile)}, batch ms
    with that choice, batch ms with the uniform starting shape)."""
    lays = ("bhw", "hwb") if layout == "any" else (layout,)
    start = None
    for lay in lays:
        cfg, times = tune_batch(frames, metric, lay, reps)
        t = min(times.values()) if times else float("inf")
        if start is None or t < start[2]:
            start = (lay, cfg, t)
    classes = sorted({int(f["bins"]) for f in frames})
    choice = {c: (start[0], start[1]) for c in classes}

    def batch_ms(ch):
        fr = [dict(f, layout=ch[int(f["bins"])][0], tile=ch[int(f["bins"])][1]) for f in frames]
        try:
            b = ih.Batch(fr, metric, layout=start[0])
        except ih.IHError:
            return float("inf")
        t = _time(lambda: b.run("phased"), reps)
        del b
        return t

    uniform_t = best_t = batch_ms(choice)
    for _ in range(rounds):
        for c in classes:
            for lay in lays:
                for cfg in batch_candidates(lay):
                    if (lay, cfg) == choice[c] or (lay == "bhw" and cfg.planes_per_wave > max(1, c)):
                        continue
                    trial = dict(choice)
                    trial[c] = (lay, cfg)
                    t = batch_ms(trial)
                    if verbose:
                        print("tune batch class %d %s %s: %.4f ms" % (c, lay, cfg, t), flush=True)
                    if t < best_t:
                        best_t, choice = t, trial
    return [choice[int(f["bins"])] for f in frames], choice, best_t, uniform_t
