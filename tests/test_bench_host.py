"""Host logic of bench.py that needs no GPU: the single-GPU guard and the
lookup of committed HBM counters, which count only for the expansion source
they were taken on."""
import json
import os
import subprocess
import sys

import bench


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(bench.REPO, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    here = bench.expand_kernel_hash()
    counters = tmp_path / "counters.json"
    counters.write_text(json.dumps({
        "current": {"source_hash": here, "bytes_per_launch": 123},
        "stale": {"source_hash": "0" * 16, "bytes_per_launch": 5},
    }))
    monkeypatch.setattr(bench, "COUNTERS", str(counters))
    assert bench.load_traffic("current") == 123
    assert bench.load_traffic("stale") is None
    assert bench.load_traffic("absent") is None
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.json"))
    assert bench.load_traffic("current") is None
    counters.write_text("not json")
    monkeypatch.setattr(bench, "COUNTERS", str(counters))
    assert bench.load_traffic("current") is None


def test_committed_counters_are_consistent():
    with open(bench.COUNTERS) as f:
        d = json.load(f)
    assert "rmat26_p8" in d  # the default workload of the bench line
    for name, ent in d.items():
        assert os.path.exists(os.path.join(bench.REPO, ent["summary"])), name
        parts = ent["fetch_bytes_per_launch"] + ent["write_bytes_per_launch"]
        assert abs(ent["bytes_per_launch"] - parts) <= 1, name
        # the kernels of one expansion step (the level kernel under its name for
        # large graphs, and the resolve of the binned push)
        assert ent["kernels"][0] in ("level_kernel", "level_kernel_wide"), name
        assert ent["kernels"][1:] == ["expand_big_kernel", "bin_resolve_kernel"], name
