"""Host-side checks of bench.py's contract (no GPU): one GPU only, and the counter
traffic constant is reported only for its own kernel class and sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_traffic_only_for_its_class_and_sources(monkeypatch):
    assert bench.measured_traffic("multidot") is None
    monkeypatch.setitem(bench.TRAFFIC, "sha256", "0" * 64)
    assert bench.measured_traffic(bench.TRAFFIC["class"]) is None
