"""Host-side logic of bench.py (no GPU): the traffic figure is taken from the
committed counter summary only for the schedule it was measured with and only
while the kernel sources are unchanged; runs on more than one GPU are refused."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_lookup_matches_schedule_and_sources():
    v = bench.measured_traffic("xinv", 3)
    assert v is None or v > 0
    assert bench.measured_traffic("xinv", 2) is None
    assert bench.measured_traffic("axial", 3) is None


def test_traffic_lookup_void_when_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "_sources_hash", lambda: "0" * 64)
    assert bench.measured_traffic("xinv", 3) is None


def test_sources_hash_is_stable_and_covers_the_kernels():
    h1 = bench._sources_hash()
    assert h1 == bench._sources_hash() and len(h1) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
