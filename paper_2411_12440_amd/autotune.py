"""Tile-shape autotuner.

Chooses the raster settings that the paper leaves open — tile shape
(tile_w x tile_h), splats staged per LDS batch, and the number of depth chunks
with the ratio between their boundaries —
by timing the whole forward + backward step on the caller's own cameras and
scene, and caches the choice in a JSON file keyed by the device, the
splat-count bucket, the resolution set, the SH degree and the settings that
change the work (kernel, lambda, AGS reading and scope, deterministic mode).
Every candidate is a configuration the library supports, and every one of
them yields the same images and gradients up to rounding order: the tile
shape changes the binning's intermediate lists, not what each pixel
composites.

Candidates are distinct launches: two settings that run the same kernels
with the same staging (for example batch 0 and batch 128 on 16x16 tiles,
where the forward kernel has 128 threads) are one candidate.  Each is timed
over `steps` individually synchronised graph replays after `warmup` ones;
the choice is by the median, and the spread (max - min over the median) is
recorded beside it.

    tuner = Autotuner()                      # cache: $LSPLAT_TUNE_CACHE or ~/.cache
    best = tuner.choose(cams, scene_off, sp, dL_dimage, sh_degree=3)
    rast = Rasterizer(cams, scene_off, sh_degree=3, **best)
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time

import torch

from .rasterizer import Rasterizer, StepGraph

# (tile_w, tile_h, batch, depth_chunks, chunk_ratio)
DEFAULT_CANDIDATES = [
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=7),
    dict(tile_w=16, tile_h=16, batch=64, depth_chunks=7),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=4),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=6, chunk_ratio=3),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5, chunk_ratio=3),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=4, chunk_ratio=3),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=1),
    dict(tile_w=16, tile_h=8, batch=64, depth_chunks=7),
    dict(tile_w=32, tile_h=8, batch=128, depth_chunks=7),
    dict(tile_w=32, tile_h=8, batch=64, depth_chunks=7),
    dict(tile_w=8, tile_h=8, batch=64, depth_chunks=7),
]


def forward_threads(tile_w: int, tile_h: int) -> int:
    """Threads of the forward kernel for a tile (two pixels per thread from
    128 pixels up): the most entries it stages per batch."""
    pix = int(tile_w) * int(tile_h)
    return pix // 2 if pix >= 128 else pix


def effective(settings: dict) -> tuple:
    """What a setting launches: tile shape, entries staged per batch by the
    forward kernel and by the one-wave backward kernel, depth chunks (0 and
    1 both build complete lists) and their boundary ratio (0 is 2; none
    without chunks)."""
    cap = forward_threads(settings["tile_w"], settings["tile_h"])
    b = int(settings.get("batch", 0)) or cap
    k = max(1, int(settings.get("depth_chunks", 1)))
    r = (int(settings.get("chunk_ratio", 0)) or 2) if k > 1 else 0
    return (int(settings["tile_w"]), int(settings["tile_h"]), min(b, cap), min(b, 64), k, r)


def distinct(candidates) -> list:
    """The candidates in order, without repeats of the same effective launch."""
    seen, out = set(), []
    for c in candidates:
        e = effective(c)
        if e not in seen:
            seen.add(e)
            out.append(dict(c))
    return out


def default_cache_path() -> str:
    return os.environ.get("LSPLAT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lsplat_tune.json"))


def tune_key(device_name: str, n_splats: int, cams, sh_degree: int, **cfg) -> str:
    """Device, splat count rounded up to a power of two, the multiset of
    image sizes, the SH degree, and the settings that change the work."""
    bucket = 1 << max(0, math.ceil(math.log2(max(1, int(n_splats)))))
    res = {}
    for w, h in zip(cams.width, cams.height):
        res[f"{int(w)}x{int(h)}"] = res.get(f"{int(w)}x{int(h)}", 0) + 1
    rs = ",".join(f"{k}*{v}" for k, v in sorted(res.items()))
    work = (f"{cfg.get('kernel', 'linear')}|lam{float(cfg.get('lambda_', 2.5)):g}"
            f"|ags{int(bool(cfg.get('ags', False)))}{int(cfg.get('ags_arg', 0))}"
            f"{int(cfg.get('ags_scope', 0))}|det{int(bool(cfg.get('deterministic', False)))}")
    return f"{device_name}|n<={bucket}|{rs}|sh{int(sh_degree)}|{work}"


class Autotuner:
    def __init__(self, cache_path: str | None = None):
        self.path = cache_path or default_cache_path()
        self.table = {}
        if os.path.exists(self.path):
            with open(self.path) as fh:
                self.table = json.load(fh)

    def lookup(self, key: str):
        hit = self.table.get(key)
        return None if hit is None else dict(hit["best"])

    def _save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def measure(self, cams, scene_off, sp, dL_dimage, sh_degree, settings, steps=10, warmup=2,
                **cfg):
        """Milliseconds of each of `steps` graph-replayed forward + backward
        steps with `settings` (one candidate), after sizing the workspace
        eagerly and `warmup` replays."""
        dev = sp["means"].device
        rast = Rasterizer(cams, scene_off, device=dev, capacity=1 << 22, sh_degree=sh_degree,
                          **settings, **cfg)
        rast.forward(sp, check_capacity=True)
        torch.cuda.synchronize(dev)
        grads = {k: torch.empty_like(v) for k, v in sp.items()}
        graph = StepGraph(rast, sp, dL_dimage, grads)
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize(dev)
        times = []
        for _ in range(steps):
            t0 = time.perf_counter()
            graph.replay()
            torch.cuda.synchronize(dev)
            times.append((time.perf_counter() - t0) * 1e3)
        if rast.overflowed():
            raise RuntimeError("workspace overflow while tuning")
        del graph, rast, grads
        return times

    def choose(self, cams, scene_off, sp, dL_dimage, sh_degree, candidates=None, steps=10,
               warmup=2, retune=False, **cfg):
        """Best settings for this workload (from the cache unless `retune`)."""
        dev = sp["means"].device
        name = torch.cuda.get_device_name(dev)
        n = int(sp["opacity"].shape[0])
        key = tune_key(name, n, cams, sh_degree, **cfg)
        if not retune:
            hit = self.lookup(key)
            if hit is not None:
                return hit
        results = []
        for cand in distinct(candidates or DEFAULT_CANDIDATES):
            times = self.measure(cams, scene_off, sp, dL_dimage, sh_degree, cand, steps, warmup,
                                 **cfg)
            med = statistics.median(times)
            results.append(dict(settings=dict(cand), ms=round(med, 4),
                                spread=round((max(times) - min(times)) / med, 4),
                                replays=len(times)))
        best = min(results, key=lambda r: r["ms"])["settings"]
        self.table[key] = dict(best=best, results=results)
        self._save()
        return dict(best)
