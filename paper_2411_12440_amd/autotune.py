"""Tile-shape autotuner.

Chooses the raster settings that the paper leaves open — tile shape
(tile_w x tile_h), splats staged per LDS batch and the number of depth chunks —
by timing the whole forward + backward step on the caller's own cameras and
scene, and caches the choice in a JSON file keyed by (device, splat-count
bucket, resolution set, SH degree).  Every candidate is a configuration the
library supports, and every one of them yields the same images and gradients
up to rounding order: the tile shape changes the binning's intermediate
lists, not what each pixel composites.

    tuner = Autotuner()                      # cache: $LSPLAT_TUNE_CACHE or ~/.cache
    best = tuner.choose(cams, scene_off, sp, dL_dimage, sh_degree=3)
    rast = Rasterizer(cams, scene_off, sh_degree=3, **best)
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from .rasterizer import Rasterizer, StepGraph

# (tile_w, tile_h, batch, depth_chunks); batch 0 stages one splat per pixel
DEFAULT_CANDIDATES = [
    dict(tile_w=16, tile_h=16, batch=0, depth_chunks=7),
    dict(tile_w=16, tile_h=16, batch=128, depth_chunks=7),
    dict(tile_w=16, tile_h=16, batch=0, depth_chunks=4),
    dict(tile_w=16, tile_h=16, batch=0, depth_chunks=1),
    dict(tile_w=16, tile_h=8, batch=0, depth_chunks=7),
    dict(tile_w=32, tile_h=8, batch=0, depth_chunks=7),
    dict(tile_w=8, tile_h=8, batch=0, depth_chunks=7),
]


def default_cache_path() -> str:
    return os.environ.get("LSPLAT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lsplat_tune.json"))


def tune_key(device_name: str, n_splats: int, cams, sh_degree: int) -> str:
    """Device, splat count rounded to a power of two, the multiset of image
    sizes, and the SH degree."""
    bucket = 1 << max(0, math.ceil(math.log2(max(1, int(n_splats)))))
    res = {}
    for w, h in zip(cams.width, cams.height):
        res[f"{int(w)}x{int(h)}"] = res.get(f"{int(w)}x{int(h)}", 0) + 1
    rs = ",".join(f"{k}*{v}" for k, v in sorted(res.items()))
    return f"{device_name}|n<={bucket}|{rs}|sh{int(sh_degree)}"


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

    def measure(self, cams, scene_off, sp, dL_dimage, sh_degree, settings, steps=3, warmup=1,
                **cfg):
        """Milliseconds per graph-replayed forward + backward step with
        `settings` (one candidate), after sizing the workspace eagerly."""
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
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if rast.overflowed():
            raise RuntimeError("workspace overflow while tuning")
        del graph, rast, grads
        return ms

    def choose(self, cams, scene_off, sp, dL_dimage, sh_degree, candidates=None, steps=3,
               warmup=1, retune=False, **cfg):
        """Best settings for this workload (from the cache unless `retune`)."""
        dev = sp["means"].device
        name = torch.cuda.get_device_name(dev)
        n = int(sp["opacity"].shape[0])
        key = tune_key(name, n, cams, sh_degree)
        if not retune:
            hit = self.lookup(key)
            if hit is not None:
                return hit
        results = []
        for cand in candidates or DEFAULT_CANDIDATES:
            ms = self.measure(cams, scene_off, sp, dL_dimage, sh_degree, cand, steps, warmup,
                              **cfg)
            results.append(dict(settings=dict(cand), ms=round(ms, 4)))
        best = min(results, key=lambda r: r["ms"])["settings"]
        self.table[key] = dict(best=best, results=results)
        self._save()
        return dict(best)
