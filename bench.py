#!/usr/bin/env python3
"""Throughput of the linear-splat rasterizer, forward + backward, on one GPU.

Workload (the paper-scale configuration): 3,200,000 splats with SH degree 3
and log-normal scales N(-4, 1), rendered into 8 cameras of 1920x1080 on a
sphere of radius 4 around the scene.  One step is the whole path over all
8 views: projection, binning (presort, scan, key generation, tile sort,
ranges), forward compositing, backward compositing and projection backward,
with a seeded N(0, 1) upstream image gradient.

Paths timed with the same kernels:
  batched   all 8 views in one call sequence (one workspace, no host sync),
            captured once in a HIP graph and replayed: the headline value
  eager     the batched sequence launched call by call with a HIP event pair
            around every kernel on its stream: per-kernel durations
  per-view  one view at a time, each with its own right-sized workspace and
            a host read-back of the intersection count after binning
The JSON line also carries the per-view rate, the dominant kernel's roofline
fraction (its algorithmic work over its average event-timed duration), the
FP64 oracle timed on a bounded sample on the host CPU, and the training-step
stages around the rasterizer on the same workload (the L1/L2/SSIM loss of
the 8 rendered views against seeded targets, one Adam step over every splat
parameter, the densification statistics and decision), each with its
algorithmic HBM bytes over its event-timed duration.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VEC_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (FMA = 2 flops)
METRIC = "Mpixel/s fwd+bwd, 3M linear splats @1080p: batched vs per-view"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--workload", type=int, default=0,
                    help="time another configuration instead of the 8-view benchmark: 1 (1k "
                         "splats, 128x128), 2 (100k SH3, 1280x720), 3 (1M, 16 uneven "
                         "cameras), 4 (3.2M, one 1920x1080 view), 5 (4 scenes, 64 cameras), "
                         "40 (the benchmark itself)")
    ap.add_argument("--splats", type=int, default=3_200_000)
    ap.add_argument("--ags", type=int, default=1)
    ap.add_argument("--depth-chunks", type=int, default=7)
    ap.add_argument("--chunk-ratio", type=int, default=0,
                    help="factor between depth-chunk boundaries with --tune 0 (0: 2)")
    ap.add_argument("--tune", type=int, default=1,
                    help="1: tile shape, LDS batch, depth chunks and their boundary ratio from "
                         "the autotuner (timed before the measurement, cached per device and "
                         "workload); 0: 16x16 tiles, --batch, --depth-chunks, --chunk-ratio")
    ap.add_argument("--batch", type=int, default=0,
                    help="LDS batch with --tune 0 (0: one splat per thread)")
    ap.add_argument("--deterministic", type=int, default=0,
                    help="1: the bitwise-reproducible backward (per-entry sums, pair sort)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-family", action="store_true",
                    help="skip the linear vs Gaussian kernel comparison")
    ap.add_argument("--no-train-stages", action="store_true",
                    help="skip the loss / Adam / densification timings")
    return ap.parse_args()


WORKLOADS = {
    1: "1k splats SH0, log-scale N(-3,0.5), one 128x128 view, fwd+bwd",
    2: "100k splats SH3, log-scale N(-3,0.5), one 1280x720 view, fwd+bwd",
    3: "1M splats SH3, 16 cameras of uneven resolution on a radius-4 sphere, fwd+bwd, batched",
    4: "3.2M splats SH3, log-scale N(-4,1), one 1920x1080 view at z=-3, fwd+bwd",
    5: "4 scenes (200k/500k/1M/2M splats SH3), 64 cameras at mixed resolutions, fwd+bwd, batched",
    40: "3.2M splats SH3, log-scale N(-4,1), 8 views 1920x1080 on a radius-4 sphere, fwd+bwd, "
        "batched",
}


def make_workload(n_splats, views):
    from paper_2411_12440_amd import scenes
    scene = scenes.make_scene(n_splats, 1004, -4.0, 1.0, 3)
    cams = scenes.sphere_cameras(views, 4.0, [(1920, 1080)] * views)
    return scene, cams


# --------------------------------------------------------------------------
# algorithmic cost of each kernel per step: what the method must move or
# compute, independent of how the kernels do it
# --------------------------------------------------------------------------

def kernel_cost(name, w):
    """(bound, amount per step, unit) for the kernels we can price.  Sort
    passes: 4 of 8 bits over the M depth keys, tile_passes over the entries."""
    N, M, n, K, Q, Qc = w["N"], w["M"], w["n_built"], w["K"], w["Q"], w["Qc"]
    tp = w["tile_passes"]
    splat_bytes = 44 + 12 * K
    if name == "tilesort_downsweep":
        return "hbm", 16.0 * n * tp, "B"
    if name == "tilesort_upsweep":
        return "hbm", 4.0 * n * tp, "B"
    if name == "presort_downsweep":
        return "hbm", 16.0 * M * 4, "B"
    if name == "presort_upsweep":
        return "hbm", 4.0 * M * 4, "B"
    if name in ("keygen", "keygen_write"):
        return "hbm", 8.0 * n + 20.0 * M, "B"
    # depth chunks: every pair is counted and written in exactly one chunk;
    # counting reads its position's pair id and rectangle and four
    # summed-area-table entries and writes a count (32 B), writing reads the
    # pair id, the rectangle and the offset (16 B) and writes 8 B per entry
    if name == "chunk_count":
        return "hbm", 32.0 * M, "B"
    if name == "chunk_write":
        return "hbm", 16.0 * M + 8.0 * n, "B"
    if name == "zero_grad2d":
        return "hbm", 72.0 * M, "B"
    if name == "project":
        return "hbm", float(splat_bytes) * N + 80.0 * M, "B"
    if name == "project_bwd":
        # centre, scale, rotation read and their gradients with the opacity's
        # written per splat; six FP64 2D-gradient fields read per pair
        return "hbm", 84.0 * N + 48.0 * M, "B"
    if name == "project_bwd_sh":
        # SH read and its gradient written, centre read and its gradient
        # updated per splat; three FP64 colour-gradient fields read per pair
        return "hbm", (24.0 * K + 36.0) * N + 24.0 * M, "B"
    # Compositing: every (pixel, splat) pair up to the pixel's last contributor
    # (Q of them) evaluates D'^2 (5 FMA = 10 flops); each contributing pair (Qc)
    # then costs 13 flops forward (sqrt, alpha, T (1 - alpha), alpha T, three
    # colour FMA) and 65 backward (alpha and T_i recovered, two 3-dot products,
    # dL/dalpha, suffix update, colour / opacity / distance / AGS weight,
    # dL/dq, the two gradient directions, mean and conic terms, and one add
    # per gradient field for the sum over pixels).  sqrt and exp count 1.
    if name == "raster_fwd":
        return "alu", 10.0 * Q + 13.0 * Qc, "flop"
    if name == "raster_bwd":
        return "alu", 10.0 * Q + 65.0 * Qc, "flop"
    return None


def source_hash(kernel):
    fname = {"raster_fwd": "raster.hip", "raster_bwd": "raster.hip", "project": "project.hip",
             "project_bwd": "project.hip"}.get(kernel, "binsort.hip")
    with open(os.path.join(ROOT, "paper_2411_12440_amd", "csrc", fname), "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()[:12]


def read_traffic(kernel):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha1") != source_hash(kernel):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# --------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on one view, across the host cores
# --------------------------------------------------------------------------

def _cpu_workers() -> int:
    """Worker processes for the oracle: the cores this process may run on,
    at most 16 (a one-GPU machine's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU = {}   # the view's oracle state, inherited by the forked workers


def _cpu_tiles(tiles):
    """Forward composite and reverse pass of the given tiles (oracle);
    seconds per tile."""
    import numpy as np

    from oracle import composite
    g = _CPU
    W, H, p = g["W"], g["H"], g["p"]
    out = []
    for t in tiles:
        t1 = time.perf_counter()
        ids = g["ids"][g["ranges"][t]:g["ranges"][t + 1]]
        ty, tx = divmod(int(t), g["gx"])
        px, py = composite._tile_pixels(tx, ty, W, H, g["cfg"])
        res = composite.composite_tile(ids, px, py, p["mean2d"], p["conic"], g["opac"], p["rgb"],
                                       g["cfg"], want_pairs=True)
        Gt = np.stack([g["G"][ch * W * H + py * W + px] for ch in range(3)], 1).astype(np.float64)
        composite.reverse_tile(res, Gt, p["mean2d"], p["conic"], g["opac"], p["rgb"], g["cfg"],
                               g["n"])
        out.append(time.perf_counter() - t1)
    return out


def _cpu_project_bwd(span):
    """Projection backward of the splats [a, b) (oracle)."""
    import numpy as np

    from oracle import projection
    g = _CPU
    a, b = span
    sub = {k: (v[a:b] if isinstance(v, np.ndarray) and v.shape[:1] == (g["n"],) else v)
           for k, v in g["p"].items()}
    n = b - a
    rs = np.random.default_rng(a)
    projection.project_backward(sub, g["sh"][a:b], g["deg"], rs.normal(size=(n, 2)),
                                rs.normal(size=(n, 3)), rs.normal(size=(n, 3)))
    return n


def cpu_baseline_child(n_splats: int, per_stratum: int = 32, strata: int = 8, seed: int = 5):
    """One 1920x1080 view of the benchmark scene through the FP64 oracle, in a
    process that has not touched the GPU (its workers are forked from it).
    Projection, FP32 binning, key generation and the (tile, depth, id) sort of
    the whole view run as the oracle runs them, on one core.  The forward and
    reverse composite of the view's tiles is measured on a stratified sample
    (strata: quantiles of the tile-list length; per_stratum tiles from each)
    spread over the worker processes, and extrapolated to every tile with the
    stratified estimator, whose standard error is reported.  The projection
    backward of every splat runs split over the workers."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import RasterConfig, binning, projection
    from oracle.render import layout
    from paper_2411_12440_amd import scenes as S

    workers = _cpu_workers()
    scene, views = make_workload(n_splats, 8)
    cams = views.subset([0])
    cfg = RasterConfig(ags=True)
    W, H = int(cams.width[0]), int(cams.height[0])
    lay = layout(np.array([0, scene.n]), cams, cfg)
    gx, gy = lay.grid[0]
    ctx = mp.get_context("fork")
    with threadpool_limits(1):
        log(f"cpu baseline: oracle on one {W}x{H} view, {workers} worker processes")
        t0 = time.perf_counter()
        p = projection.project(scene.means, scene.scales, scene.quats, scene.sh, scene.sh_degree,
                               cams.viewmat[0], cams.intrin[0], W, H, cfg)
        rect, nt, dk = binning.binning_fp32(scene.means, scene.scales, scene.quats,
                                            cams.viewmat[0], cams.intrin[0], W, H, cfg)
        t_proj = time.perf_counter() - t0
        t0 = time.perf_counter()
        g_, d_, i_ = binning.intersections_array(rect, nt, dk, np.arange(scene.n), 0, gx)
        g_, d_, i_ = binning.sort_arrays(g_, d_, i_)
        ranges = binning.tile_ranges(g_, gx * gy)
        t_sort = time.perf_counter() - t0
        n_isect = int(len(i_))
        del g_, d_, rect, nt, dk
        log(f"cpu baseline: projection + binning {t_proj:.1f} s, keys + sort of {n_isect} "
            f"intersections {t_sort:.1f} s")
        # stratified sample of tiles by list length
        lens = np.diff(ranges)
        edges = np.quantile(lens, np.linspace(0.0, 1.0, strata + 1))
        stratum = np.clip(np.searchsorted(edges[1:-1], lens, side="right"), 0, strata - 1)
        rs = np.random.default_rng(seed)
        sample, of = [], []
        for h in range(strata):
            members = np.nonzero(stratum == h)[0]
            k = min(per_stratum, len(members))
            sample += [int(t) for t in rs.choice(members, k, replace=False)]
            of += [h] * k
        _CPU.update(W=W, H=H, p=p, ids=i_, ranges=ranges, gx=gx, cfg=cfg,
                    opac=scene.opacity.astype(np.float64), n=scene.n,
                    G=S.upstream_grad(cams, 7004), sh=scene.sh, deg=scene.sh_degree)
        chunks = [sample[j::workers] for j in range(workers)]
        spans = np.linspace(0, scene.n, 4 * workers + 1).astype(np.int64)
        with ctx.Pool(workers) as pool:
            t0 = time.perf_counter()
            times = pool.map(_cpu_tiles, chunks)
            wall = time.perf_counter() - t0
            t0 = time.perf_counter()
            pool.map(_cpu_project_bwd, list(zip(spans[:-1], spans[1:])))
            t_pbwd = time.perf_counter() - t0
    per = np.zeros(len(sample))
    for j in range(workers):
        per[j::workers] = times[j]
    of = np.array(of)
    est, var = 0.0, 0.0
    for h in range(strata):
        Nh = int(np.sum(stratum == h))
        x = per[of == h]
        est += Nh * float(x.mean())
        if len(x) > 1:
            var += Nh * Nh * (1.0 - len(x) / Nh) * float(x.var(ddof=1)) / len(x)
    # the tiles' seconds over the workers, at the parallel efficiency the
    # sample itself reached
    eff = wall / (float(per.sum()) / workers)
    t_tiles = est / workers * eff
    rel_se = math.sqrt(var) / est
    per_view = t_proj + t_sort + t_tiles + t_pbwd
    mpx = W * H / per_view / 1e6
    sample_txt = (
        f"one {W}x{H} view of the {scene.n}-splat scene (the first of the 8 views), FP64 oracle: "
        f"projection + FP32 binning of every splat {t_proj:.1f} s and key generation + sort of its "
        f"{n_isect} intersections {t_sort:.1f} s, one core each as the oracle runs them; forward + "
        f"reverse composite of a stratified sample of {len(sample)} of the {gx * gy} tiles "
        f"({strata} strata by list length) over {workers} processes, {wall:.1f} s wall for "
        f"{per.sum():.1f} s of tile time, extrapolated to every tile: {t_tiles:.1f} s (relative "
        f"standard error of the extrapolation {rel_se:.1%}); projection backward of every splat "
        f"over {workers} processes {t_pbwd:.1f} s; {per_view:.1f} s per view")
    return dict(value=round(mpx, 6), unit="Mpixel/s", cores=workers, kind="oracle",
                cpu_model=_cpu_model(), nproc=os.cpu_count(), rel_std_error=round(rel_se, 4),
                seconds_per_view=round(per_view, 2), sample=sample_txt)


def cpu_baseline(n_splats: int):
    """Runs cpu_baseline_child in a fresh interpreter (this process holds the
    GPU; its forked children must not) and returns its record."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                        str(n_splats)], stdout=subprocess.PIPE, text=True, timeout=1200)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline child failed with status {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])


# --------------------------------------------------------------------------

def training_stages(B, S, torch, rast, sp, grads, cams, steps, warmup):
    """Event-timed loss, Adam and densification calls on the step's own
    outputs, with algorithmic bytes: loss 12 B per pixel and channel (image
    and target read, gradient written), Adam 28 B per parameter (parameter,
    gradient and both moments read; parameter and moments written),
    statistics 44 B per visible-or-not pair (two FP64 gradient components,
    the tile count, the FP64 conic) plus 24 B per splat (accumulators read
    and written), decision 29 B per splat."""
    dev = rast.image.device
    N = int(sp["opacity"].numel())
    M = int(rast.layout.n_pairs)
    P = int(rast.layout.n_pixels)
    _, target = S.image_pair(cams.width, cams.height, seed=7100)
    target = torch.from_numpy(target).to(dev)
    lws = torch.empty(B.ls_loss_workspace_size(rast.cams), dtype=torch.uint8, device=dev)
    dimg = torch.empty_like(rast.image)
    lossv = torch.empty(cams.n, dtype=torch.float64, device=dev)
    state = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in sp.items()}
    params = {k: v.clone() for k, v in sp.items()}
    lrs = dict(means=1.6e-4, scales=5e-3, quats=1e-3, opacity=5e-2, sh=2.5e-3)
    acc_g = torch.zeros(N, dtype=torch.float32, device=dev)
    acc_c = torch.zeros(N, dtype=torch.int32, device=dev)
    acc_e = torch.zeros(N, dtype=torch.float32, device=dev)
    acc = B.densify_acc(acc_g, acc_c, acc_e)
    action = torch.empty(N, dtype=torch.uint8, device=dev)
    counts = torch.empty(3, dtype=torch.int64, device=dev)
    dprm = B.densify_params(1.0)

    def run(t):
        B.ls_loss(rast.cams, rast.image, target, dimg, lossv, lws)
        for k in params:
            B.ls_adam(B.adam_params(lrs[k], t), params[k], grads[k], *state[k])
        B.ls_densify_stats(rast.cfg, rast.cams, rast.ws, rast.capacity, acc)
        B.ls_densify_select(dprm, N, params["scales"], params["opacity"], acc, action, counts)

    for t in range(1, warmup + 1):
        run(t)
    torch.cuda.synchronize()
    B.ls_profile_read(reset=True)
    B.ls_profile_enable(True)
    for t in range(warmup + 1, warmup + steps + 1):
        run(t)
    torch.cuda.synchronize()
    B.ls_profile_enable(False)
    kt = {n: (c, t) for n, c, t in B.ls_profile_read(reset=True)}
    n_params = sum(int(v.numel()) for v in sp.values())
    cost = {"loss": 12.0 * 3 * P, "adam": 28.0 * n_params,
            "densify_stats": 44.0 * M + 24.0 * N, "densify_select": 29.0 * N}
    out = {}
    for name, amount in cost.items():
        if name not in kt:
            continue
        ms = kt[name][1] / steps
        gbs = amount / (ms * 1e-3) / 1e9
        out[name] = dict(ms=round(ms, 4), algorithmic_bytes=amount, achieved_gbs=round(gbs, 1),
                         frac=round(gbs / HBM_PEAK_GBS, 4))
    out["loss_per_view"] = [round(float(x), 6) for x in lossv.cpu().tolist()]
    out["densify_counts"] = counts.cpu().tolist()
    out["note"] = ("per call over the 8-view step; Adam over all %d parameters in 5 groups; "
                   "algorithmic bytes as in bench.training_stages" % n_params)
    del lws, dimg, state, params
    return out


def main():
    if len(sys.argv) == 2 and sys.argv[1] == "--copy-calibration":
        # a plain device-to-device copy of 1 GiB, three times: the reference
        # against which the HBM counters (FETCH_SIZE, WRITE_SIZE) are scaled
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return
    if len(sys.argv) == 3 and sys.argv[1] == "--cpu-baseline-child":
        # the oracle baseline in a process of its own that never touches the GPU
        print(json.dumps(cpu_baseline_child(int(sys.argv[2]))), flush=True)
        return
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this rasterizer runs on one GPU.  Across GPUs the views would be "
              "sharded, with one all-reduce of the splat gradients per step; that path is not "
              "built, so only --gpus 1 runs.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2411_12440_amd import binding as B
    from paper_2411_12440_amd.rasterizer import Rasterizer, StepGraph, scene_to_device
    from paper_2411_12440_amd import scenes as S

    dev = torch.device("cuda:0")
    if args.workload:
        log(f"bench: building workload {args.workload}")
        scene, off, cams = S.workload(args.workload)
        off = np.asarray(off, np.int64)
        workload_name = WORKLOADS[args.workload]
    else:
        log(f"bench: building workload ({args.splats} splats, {args.views} views)")
        scene, cams = make_workload(args.splats, args.views)
        off = np.array([0, scene.n])
        workload_name = WORKLOADS[40]
    sp = scene_to_device(scene, dev)
    G_all = torch.from_numpy(S.upstream_grad(cams, 7004)).to(dev)
    settings = dict(tile_w=16, tile_h=16, batch=args.batch, depth_chunks=args.depth_chunks,
                    chunk_ratio=args.chunk_ratio)
    tuned = None
    if args.tune:
        from paper_2411_12440_amd import autotune
        log("bench: autotuning tile shape, LDS batch, depth chunks and their ratio")
        tuner = autotune.Autotuner()
        settings = tuner.choose(cams, off, sp, G_all, 3, ags=bool(args.ags),
                                deterministic=bool(args.deterministic))
        tuned = tuner.table.get(autotune.tune_key(torch.cuda.get_device_name(dev), scene.n,
                                                  cams, 3, ags=bool(args.ags),
                                                  deterministic=bool(args.deterministic)))
        log(f"bench: tuned settings {settings}")
    cfgkw = dict(sh_degree=scene.sh_degree, ags=bool(args.ags),
                 deterministic=bool(args.deterministic), **settings)
    from paper_2411_12440_amd.autotune import effective
    eff = effective(settings)
    P = int(sum(int(w) * int(h) for w, h in zip(cams.width, cams.height)))

    # ---- batched path -------------------------------------------------------
    log("bench: sizing the batched workspace")
    rast = Rasterizer(cams, off, device=dev, capacity=1 << 24, **cfgkw)
    rast.forward(sp, check_capacity=True)
    torch.cuda.synchronize()
    n_isect = rast.n_isect()
    n_built = rast.n_built()
    rast._alloc(max(int(n_built * 1.05) + 4096, n_isect // 12))
    grads = {k: torch.empty_like(v) for k, v in sp.items()}

    def step_batched():
        rast.project(sp)
        rast.bin_sort()
        rast.rasterize_fwd()
        rast.rasterize_bwd(sp, G_all, grads)

    # headline: the whole step captured once in a HIP graph, replayed
    log("bench: capturing the batched step in a HIP graph")
    graph = StepGraph(rast, sp, G_all, grads)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} graph replays (n_isect={n_isect})")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / args.steps
    assert not rast.overflowed()
    # the same kernels launched eagerly, each bracketed by HIP events on its
    # stream, for per-kernel durations
    for _ in range(args.warmup):
        step_batched()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} eager batched steps with kernel events")
    B.ls_profile_read(reset=True)
    B.ls_profile_enable(True)
    e0.record()
    for _ in range(args.steps):
        step_batched()
    e1.record()
    torch.cuda.synchronize()
    B.ls_profile_enable(False)
    ms_eager = e0.elapsed_time(e1) / args.steps
    ktimes = B.ls_profile_read(reset=True)
    assert not rast.overflowed()
    last = rast.last.to(torch.int64)
    Q = int(last.sum().item())
    Qc = rast.contributions()
    chunk_entries = [int(v) for v in np.diff(rast.lists()[0])]
    value = P / (ms_batched * 1e-3) / 1e6
    log(f"bench: batched {ms_batched:.3f} ms/step, {value:.1f} Mpx/s")

    # ---- per-view path ------------------------------------------------------
    per_view = None
    if not args.no_per_view:
        views = []
        pix_off = 0
        for c in range(cams.n):
            one = cams.subset([c])
            r = Rasterizer(one, off, device=dev, capacity=1 << 24, **cfgkw)
            r.forward(sp, check_capacity=True)
            torch.cuda.synchronize()
            r._alloc(max(int(r.n_built() * 1.05) + 4096, r.n_isect() // 12))
            npx = int(cams.width[c]) * int(cams.height[c])
            g_v = G_all[3 * pix_off: 3 * (pix_off + npx)]
            pix_off += npx
            views.append((r, g_v, {k: torch.empty_like(v) for k, v in sp.items()}))

        def step_per_view():
            for r, g_v, gr in views:
                r.project(sp)
                r.bin_sort()
                r.n_isect()                         # host read-back, as a per-view loop does
                r.rasterize_fwd()
                if r.overflowed():
                    raise RuntimeError("per-view capacity overflow")
                r.rasterize_bwd(sp, g_v, gr)

        for _ in range(args.warmup):
            step_per_view()
        torch.cuda.synchronize()
        log(f"bench: timing {args.steps} per-view steps")
        e0.record()
        for _ in range(args.steps):
            step_per_view()
        e1.record()
        torch.cuda.synchronize()
        ms_pv = e0.elapsed_time(e1) / args.steps
        per_view = dict(value=round(P / (ms_pv * 1e-3) / 1e6, 3), ms_per_step=round(ms_pv, 3),
                        batched_over_per_view=round(ms_pv / ms_batched, 3))
        log(f"bench: per-view {ms_pv:.3f} ms/step, ratio {ms_pv / ms_batched:.3f}")
        del views

    # ---- kernel family: the same step with the Gaussian kernel ------------------
    family = None
    if not args.no_family:
        def time_kernel(kname, lam):
            kw = dict(cfgkw, kernel=kname, lambda_=lam, ags=False)
            r = Rasterizer(cams, off, device=dev, capacity=1 << 24, **kw)
            r.forward(sp, check_capacity=True)
            torch.cuda.synchronize()
            r._alloc(max(int(r.n_built() * 1.05) + 4096, r.n_isect() // 12))
            gr = {k: torch.empty_like(v) for k, v in sp.items()}
            gph = StepGraph(r, sp, G_all, gr)
            for _ in range(args.warmup):
                gph.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                gph.replay()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps

            def eager():
                r.project(sp)
                r.bin_sort()
                r.rasterize_fwd()
                r.rasterize_bwd(sp, G_all, gr)

            eager()
            torch.cuda.synchronize()
            B.ls_profile_read(reset=True)
            B.ls_profile_enable(True)
            for _ in range(args.steps):
                eager()
            torch.cuda.synchronize()
            B.ls_profile_enable(False)
            kt = {n: t / args.steps for n, _, t in B.ls_profile_read(reset=True)}
            assert not r.overflowed()
            res = dict(lambda_=lam, ms_per_step=round(ms, 3),
                       value=round(P / (ms * 1e-3) / 1e6, 3),
                       raster_fwd_ms=round(kt.get("raster_fwd", 0.0), 3),
                       raster_bwd_ms=round(kt.get("raster_bwd", 0.0), 3),
                       entries_built=int(r.n_built()), contributing_pairs=int(r.contributions()))
            del gph, r, gr
            return res

        log("bench: kernel family (linear without AGS, Gaussian)")
        family = {"linear": time_kernel("linear", 2.5), "gaussian": time_kernel("gaussian", 1.0)}
        family["note"] = ("same scene, cameras and step, both without AGS (defined for the linear "
                          "kernel only); linear lambda 2.5, Gaussian lambda 1 with the 3-sigma cut")
        log(f"bench: family {family}")

    train = None
    if not args.no_train_stages:
        log("bench: training-step stages (loss, Adam, densification)")
        step_batched()
        torch.cuda.synchronize()
        train = training_stages(B, S, torch, rast, sp, grads, cams, args.steps, args.warmup)
        log(f"bench: training stages {train}")

    # ---- roofline of the dominant kernel --------------------------------------
    T_tiles = int(rast.layout.n_tiles)
    tile_passes = max(1, ((T_tiles - 1).bit_length() + 7) // 8)
    w = dict(N=scene.n, M=int(rast.layout.n_pairs), n_isect=n_isect, n_built=n_built,
             K=(scene.sh_degree + 1) ** 2, Q=Q, Qc=Qc, tile_passes=tile_passes)
    kernels = []
    for name, launches, total in ktimes:
        row = dict(kernel=name, launches=launches, avg_ms=round(total / launches, 4),
                   total_ms_per_step=round(total / args.steps, 4))
        cost = kernel_cost(name, w)
        if cost is not None:       # fraction of its roofline over the step
            bound, amount, _ = cost
            rate = amount / (total / args.steps * 1e-3)
            row["frac"] = round(rate / (HBM_PEAK_GBS * 1e9 if bound == "hbm"
                                        else FP64_VEC_PEAK_TFLOPS * 1e12), 4)
        kernels.append(row)
    # whole pipeline: each priced kernel's floor (its algorithmic work at the
    # chip's peak rate) summed over the step, against the measured step
    floor_ms = priced_ms = 0.0
    for row in kernels:
        cost = kernel_cost(row["kernel"], w)
        if cost is None:
            continue
        bound, amount, _ = cost
        floor_ms += 1e3 * amount / (HBM_PEAK_GBS * 1e9 if bound == "hbm"
                                    else FP64_VEC_PEAK_TFLOPS * 1e12)
        priced_ms += row["total_ms_per_step"]
    kernel_ms = sum(r["total_ms_per_step"] for r in kernels)
    pipeline = dict(floor_ms=round(floor_ms, 4), step_ms=round(ms_batched, 4),
                    frac=round(floor_ms / ms_batched, 4),
                    priced_kernel_ms=round(priced_ms, 4),
                    unpriced_kernel_ms=round(kernel_ms - priced_ms, 4),
                    note="sum over the priced kernels of algorithmic work at peak (HBM 8 TB/s, "
                         "FP64 vector 78.6 TFLOP/s) over the graph-replayed step; the unpriced "
                         "kernels (scans, ranges, list bookkeeping) count as time with no floor")
    roof = None
    if kernels:
        dom = kernels[0]
        cost = kernel_cost(dom["kernel"], w)
        if cost is not None:
            bound, amount, unit = cost
            launches_per_step = dom["launches"] / args.steps
            per_launch = amount / launches_per_step
            sec = dom["avg_ms"] * 1e-3
            if bound == "hbm":
                achieved = per_launch / sec / 1e9
                peak, u = HBM_PEAK_GBS, "GB/s"
            else:
                achieved = per_launch / sec / 1e12
                peak, u = FP64_VEC_PEAK_TFLOPS, "TFLOP/s"
            roof = dict(kernel=dom["kernel"], bound=bound, achieved=round(achieved, 3), peak=peak,
                        unit=u, frac=round(achieved / peak, 4),
                        traffic=read_traffic(dom["kernel"]),
                        algorithmic_per_launch=per_launch, avg_launch_ms=dom["avg_ms"])

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on one view (host CPU, worker processes)")
        cpu = cpu_baseline(args.splats)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": workload_name,
                   "views": cams.n, "pixels_per_step": P, "n_isect": n_isect,
                   "entries_built": n_built, "depth_chunks": settings["depth_chunks"],
                   "chunk_ratio": int(settings.get("chunk_ratio", 0)) or 2,
                   "chunk_entries": chunk_entries,
                   "pairs_to_last": Q, "contributing_pairs": Qc, "ags": bool(args.ags),
                   "deterministic": bool(args.deterministic),
                   "tile": f"{settings['tile_w']}x{settings['tile_h']}",
                   "lds_batch": settings["batch"],
                   "staged_per_batch": {"forward": eff[2], "backward": eff[3]},
                   "autotuned": bool(args.tune),
                   "tuning": None if tuned is None else tuned.get("results"),
                   "parallelism": "single GPU"},
        "eager": {"ms_per_step": round(ms_eager, 4),
                  "value": round(P / (ms_eager * 1e-3) / 1e6, 3),
                  "note": "same step launched eagerly with an event pair around every kernel"},
        "per_view": per_view,
        "kernel_family": family,
        "training_stages": train,
        "roofline": roof,
        "pipeline": pipeline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
