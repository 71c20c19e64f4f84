"""bench.py's host-side contract, without a GPU: a request for more than one
GPU is refused with a message, and the counter-derived fields (scatter
traffic, whole-pass bytes) are reported only while the kernel sources are
the ones the committed counters were taken with."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_fields_follow_the_kernel_sources(monkeypatch):
    with open(bench.PMC_FILE) as f:
        pmc = json.load(f)
    n = pmc["n"]
    if pmc.get("kernel_source_sha") != bench.kernel_source_sha():
        pytest.skip("the committed counters predate the current kernel sources")
    traffic = bench.measured_traffic(n)
    assert traffic == pmc["hbm_bytes_per_launch"]
    # traffic within a few percent of the algorithmic 16 B per pair: no re-reads
    assert 1.0 <= traffic / (16 * n) < 1.1
    pass_bytes = bench.measured_pass_bytes(n)
    assert pass_bytes > traffic
    assert bench.measured_traffic(n + 1) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.measured_traffic(n) is None
    assert bench.measured_pass_bytes(n) is None
