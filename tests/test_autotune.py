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
    assert k == "dev|n<=4194304|1920x1080*2,640x480*1|sh3"
    assert at.tune_key("dev", 4_194_304, cams, 3) == k
    assert at.tune_key("dev", 4_194_305, cams, 3) != k
    cams2 = scenes.sphere_cameras(3, 4.0, [(640, 480), (1920, 1080), (1920, 1080)])
    assert at.tune_key("dev", 3_000_000, cams2, 3) == k


def test_choose_takes_the_fastest_and_caches(tmp_path, monkeypatch):
    at = _tuner_module()
    fake_ms = {(16, 16, 0, 7): 5.0, (16, 8, 0, 7): 3.0, (8, 8, 0, 7): 4.0}
    calls = []

    def measure(self, cams, off, sp, dL, deg, s, steps=3, warmup=1, **cfg):
        calls.append(s)
        return fake_ms[(s["tile_w"], s["tile_h"], s["batch"], s["depth_chunks"])]

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
    # a new tuner reads the cache and measures nothing
    t2 = at.Autotuner(str(path))
    assert t2.choose(cams, np.array([0, 1000]), sp, None, 0, candidates=cands) == best
    assert len(calls) == 3


class _FakeTensor:
    device = "cpu"
