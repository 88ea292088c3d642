"""Host-side logic of bench.py (no GPU): a counter figure is taken from the
committed summary only for the schedule it was measured with and only while the
kernel's sources are unchanged; runs on more than one GPU are refused."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary(tmp_path, hashes, rows):
    lines = [f"sources_sha256 {k}: {h}" for k, h in hashes.items()] + rows
    p = tmp_path / "traffic.md"
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def test_traffic_lookup_matches_schedule_and_sources(tmp_path, monkeypatch):
    hashes = {k: bench._sources_hash(k) for k in bench.KERNEL_SOURCES}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, hashes, [
        "traffic_bytes_per_launch axial sched 0: 1.5e8",
        "traffic_bytes_per_iteration: 2.2e9"]))
    assert bench.measured_traffic("axial", 0) == 1.5e8
    assert bench.measured_traffic("axial", 1) is None
    assert bench.measured_traffic("xinv", 0) is None
    assert bench.measured_iteration_traffic() == 2.2e9


def test_traffic_lookup_void_when_sources_change(tmp_path, monkeypatch):
    hashes = {k: bench._sources_hash(k) for k in bench.KERNEL_SOURCES}
    hashes["axial"] = "0" * 64
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, hashes, [
        "traffic_bytes_per_launch axial sched 0: 1.5e8",
        "traffic_bytes_per_iteration: 2.2e9"]))
    assert bench.measured_traffic("axial", 0) is None
    assert bench.measured_iteration_traffic() is None


def test_sources_hash_is_stable_and_covers_the_kernels():
    for k in bench.KERNEL_SOURCES:
        h1 = bench._sources_hash(k)
        assert h1 == bench._sources_hash(k) and len(h1) == 64
    assert bench._sources_hash("axial") != bench._sources_hash("xinv")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
