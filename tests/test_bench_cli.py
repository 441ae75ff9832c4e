"""Host-side contract of bench.py (no GPU): one GPU only, the workload
table, and the committed HBM-traffic records it reads."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_table_names_the_three_workloads():
    assert sorted(bench.WORKLOADS) == ["sweep", "tree", "tube"]
    for name, (tag, text) in bench.WORKLOADS.items():
        assert tag.startswith(name)
        assert "elastic" in text and "tau=0.8" in text


@pytest.mark.parametrize("tag", ["tree", "sweep64"])
def test_committed_traffic_records_are_well_formed(tag):
    """Each record holds FETCH_SIZE / WRITE_SIZE per dispatch for FP32 and
    FP16 storage, scaled by the copy reference (fetch x2, write x1), and the
    bytes per launch agree with those counters."""
    d = json.load(open(os.path.join(ROOT, "profiles", f"update_kernel_{tag}_traffic.json")))
    assert len(d["kernel_hash"]) == 16
    for dt in ("f32", "f16"):
        e = d["per_dtype"][dt]
        total = e["fetch_kib"] * 1024 * d["scale"]["fetch"] + e["write_kib"] * 1024 * d["scale"]["write"]
        assert abs(total - e["bytes_per_launch"]) <= 1e-6 * total + 1024
        # reads and writes at least the populations once (2 x 19 x s per site)
        s = {"f32": 4, "f16": 2}[dt]
        assert e["bytes_per_site"]["write"] >= 19 * s - 0.01
        assert e["bytes_per_site"]["fetch"] >= 19 * s - 0.01


def test_traffic_lookup_follows_the_kernel_hash(tmp_path, monkeypatch):
    rec = {"kernel_hash": "0" * 16, "per_dtype": {"f32": {"bytes_per_launch": 123}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "update_kernel_tube32_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.traffic_from_profiles("f32") == 123
    assert bench.traffic_from_profiles("f16") is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "1" * 16)
    assert bench.traffic_from_profiles("f32") is None
