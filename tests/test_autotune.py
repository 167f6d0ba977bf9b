"""Host logic of the tile-shape autotuner: cache keys, the choice of the
fastest candidate, and the JSON cache round trip (timings are stubbed; the
GPU test runs the real measurement)."""
from __future__ import annotations

import json

import numpy as np
import pytest

from paper_2411_12440_amd import scenes


def _tuner_module():
    try:
        from paper_2411_12440_amd import autotune
    except ImportError as e:        # library not built
        pytest.skip(str(e))
    return autotune


def test_key_buckets_and_resolution_multiset():
    at = _tuner_module()
    cams = scenes.sphere_cameras(3, 4.0, [(1920, 1080), (640, 480), (1920, 1080)])
    k = at.tune_key("dev", 3_000_000, cams, 3)
    assert k == "dev|n<=4194304|1920x1080*2,640x480*1|sh3|linear|lam2.5|ags000|det0"
    assert at.tune_key("dev", 4_194_304, cams, 3) == k
    assert at.tune_key("dev", 4_194_305, cams, 3) != k
    cams2 = scenes.sphere_cameras(3, 4.0, [(640, 480), (1920, 1080), (1920, 1080)])
    assert at.tune_key("dev", 3_000_000, cams2, 3) == k
    # the settings that change the work are part of the key
    others = [dict(ags=True), dict(ags=True, ags_scope=1), dict(kernel="gaussian", lambda_=1.0),
              dict(deterministic=True)]
    keys = {at.tune_key("dev", 3_000_000, cams, 3, **o) for o in others}
    assert len(keys) == len(others) and k not in keys


def test_candidates_are_distinct_launches():
    """Batch 0 and the forward kernel's thread count stage the same entries;
    every default candidate is a different launch and a valid setting."""
    at = _tuner_module()
    from paper_2411_12440_amd import binding as B
    assert at.effective(dict(tile_w=16, tile_h=16, batch=0, depth_chunks=7)) == \
        at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=7))
    assert at.effective(dict(tile_w=16, tile_h=16, batch=64, depth_chunks=7)) != \
        at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=7))
    assert at.effective(dict(tile_w=16, tile_h=8, batch=0, depth_chunks=7))[2] == 64
    # the chunk boundary ratio: 0 is 2, and it changes nothing without chunks
    assert at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5, chunk_ratio=0)) == \
        at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5, chunk_ratio=2))
    assert at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5, chunk_ratio=3)) != \
        at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=5))
    assert at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=1, chunk_ratio=3)) == \
        at.effective(dict(tile_w=16, tile_h=16, batch=128, depth_chunks=1))
    assert len(at.distinct(at.DEFAULT_CANDIDATES)) == len(at.DEFAULT_CANDIDATES)
    dup = at.DEFAULT_CANDIDATES + [dict(tile_w=16, tile_h=16, batch=0, depth_chunks=7)]
    assert at.distinct(dup) == at.DEFAULT_CANDIDATES
    cams = B.CamerasHost(None, None, np.array([64]), np.array([48]), np.zeros(1), np.array([0, 10]))
    for c in at.DEFAULT_CANDIDATES:
        assert B.ls_workspace_size(B.make_config(**c), cams, 0) > 0


def test_choose_takes_the_fastest_and_caches(tmp_path, monkeypatch):
    at = _tuner_module()
    fake_ms = {(16, 16, 0, 7): 5.0, (16, 8, 0, 7): 3.0, (8, 8, 0, 7): 4.0}
    calls = []

    def measure(self, cams, off, sp, dL, deg, s, steps=10, warmup=2, **cfg):
        calls.append(s)
        m = fake_ms[(s["tile_w"], s["tile_h"], s["batch"], s["depth_chunks"])]
        return [m * (1.0 + 0.01 * (i % 3 - 1)) for i in range(steps)]

    monkeypatch.setattr(at.Autotuner, "measure", measure)
    monkeypatch.setattr(at.torch.cuda, "get_device_name", lambda dev=None: "fake-gpu")
    cands = [dict(tile_w=w, tile_h=h, batch=b, depth_chunks=k) for (w, h, b, k) in fake_ms]
    sp = {"means": _FakeTensor(), "opacity": np.zeros(1000)}
    cams = scenes.front_camera(64, 48)
    path = tmp_path / "tune.json"
    t = at.Autotuner(str(path))
    best = t.choose(cams, np.array([0, 1000]), sp, None, 0, candidates=cands)
    assert best == dict(tile_w=16, tile_h=8, batch=0, depth_chunks=7)
    assert len(calls) == 3
    table = json.loads(path.read_text())
    (key, entry), = table.items()
    assert key.startswith("fake-gpu|n<=1024|64x48*1|sh0")
    assert [r["ms"] for r in entry["results"]] == [5.0, 3.0, 4.0]
    assert [r["replays"] for r in entry["results"]] == [10, 10, 10]
    assert all(abs(r["spread"] - 0.02) < 1e-9 for r in entry["results"])
    # a new tuner reads the cache and measures nothing
    t2 = at.Autotuner(str(path))
    assert t2.choose(cams, np.array([0, 1000]), sp, None, 0, candidates=cands) == best
    assert len(calls) == 3


class _FakeTensor:
    device = "cpu"
