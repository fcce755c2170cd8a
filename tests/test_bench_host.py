"""Host-side logic of bench.py: the kernel a tile shape launches, the counted-
traffic lookup (only for matching kernel sources), and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.fixture(scope="module")
def lbm():
    from paper_2504_10539_amd import lbm as L
    return L


def test_kernel_names(lbm):
    tiles = lbm.tiles()
    strip = next(t for t in tiles if not t["paired"] and t["threads"] == 512 and t["cells"] == 1)
    pair = next(t for t in tiles if t["paired"] and t["threads"] == 256)
    assert bench.kernel_name(lbm, strip["id"], lbm.LBM_F32) == \
        f"k_step<StoreF32, 512, 1, {strip['prefetch']}>"
    assert bench.kernel_name(lbm, pair["id"], lbm.LBM_F16_SHIFTED) == \
        f"k_step_pair<StoreF16S, 4, {pair['prefetch']}>"
    two = next(t for t in tiles if t["steps"] == 2 and t["threads"] == 256)
    assert bench.kernel_name(lbm, two["id"], lbm.LBM_F16_CELL) == \
        f"k_step2<StoreF16C, 256, {two['prefetch']}, {two['width']}>"


def test_launch_figures_count_one_read_and_write_per_launch(lbm):
    tiles = lbm.tiles()
    one = next(t for t in tiles if t["steps"] == 1)
    two = next(t for t in tiles if t["steps"] == 2)
    a = bench.launch_figures(lbm, one["id"], 0.1, 72, 1000)
    b = bench.launch_figures(lbm, two["id"], 0.1, 72, 1000)
    assert a["steps_per_launch"] == 1 and b["steps_per_launch"] == 2
    assert a["launch_ms"] == pytest.approx(0.1) and b["launch_ms"] == pytest.approx(0.2)
    assert a["achieved_gbs"] == pytest.approx(72 * 1000 / 1e-4 / 1e9)
    assert b["achieved_gbs"] == pytest.approx(a["achieved_gbs"] / 2)


def test_traffic_lookup_requires_matching_sources(lbm, tmp_path, monkeypatch):
    t = next(t for t in lbm.tiles() if not t["paired"] and t["threads"] == 256)
    entry = {"storage": "f32", "n": 512, "kernel": bench.kernel_name(lbm, t["id"], lbm.LBM_F32),
             "width": t["width"], "rows": t["rows"], "bytes_per_launch": 12345,
             "kernel_hash": "abc"}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "step_counters.json").write_text(json.dumps({"entries": [entry]}))
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.traffic_from_profiles(lbm, "abc", "f32", 512, t["id"]) == 12345
    assert bench.traffic_from_profiles(lbm, "other", "f32", 512, t["id"]) is None
    assert bench.traffic_from_profiles(lbm, "abc", "f32", 1024, t["id"]) is None


def test_committed_counters_name_real_shapes(lbm):
    with open(os.path.join(ROOT, "profiles", "step_counters.json")) as fh:
        d = json.load(fh)
    # balanced shapes (rows 0) take a height per grid and device
    shapes = {(bench.kernel_name(lbm, t["id"], s), t["width"], t["rows"])
              for t in lbm.tiles()
              for s in (lbm.LBM_F32, lbm.LBM_F16_SHIFTED, lbm.LBM_F16_CELL, lbm.LBM_F16_MOMENT)}
    assert d["entries"]
    for e in d["entries"]:
        assert ((e["kernel"], e["width"], e["rows"]) in shapes
                or ((e["kernel"], e["width"], 0) in shapes and 2 <= e["rows"] <= 256)), e
        bpu = {"f32": 72, "f16_shifted": 36, "f16_cell": 40, "f16_moment": 48}[e["storage"]]
        assert e["bytes_per_launch"] > 0.9 * bpu * e["n"] ** 2


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
