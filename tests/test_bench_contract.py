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
    path = bench.pmc_file("uniform_u32_pairs")
    with open(path) as f:
        pmc = json.load(f)
    n = pmc["n"]
    if pmc.get("kernel_source_sha") != bench.kernel_source_sha():
        pytest.skip("the committed counters predate the current kernel sources")
    traffic = bench.measured_traffic(n)
    assert traffic == sum(v["bytes_per_dispatch"] for k, v in pmc["kernels"].items()
                          if k.startswith("rs::rs_rank_scatter"))
    # traffic within a few percent of the algorithmic 16 B per pair: no re-reads
    assert 1.0 <= traffic / (16 * n) < 1.1
    pass_bytes = bench.measured_pass_bytes(n)
    assert pass_bytes > traffic
    assert bench.measured_traffic(n + 1) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.measured_traffic(n) is None
    assert bench.measured_pass_bytes(n) is None


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path):
    """Counter values per dispatch are averaged per kernel, scaled so that
    the calibration copy reads 1 GiB and writes 1 GiB, and summed over the
    library's kernels into bytes per sort; other kernels are left out."""
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    cal = "void at::native::vectorized_elementwise_kernel<bitwise_not_kernel>"
    fetch = head + "".join([
        f"1,{cal},FETCH_SIZE,524288\n", f"2,{cal},FETCH_SIZE,524288\n",
        "3,void rs::rs_tile_histogram<x>(int),FETCH_SIZE,1000\n", "4,rs::rs_tile_histogram<x>,FETCH_SIZE,3000\n",
        '5,"void rs::rs_rank_scatter<y, 2>(rs::P<a>, int)",FETCH_SIZE,500\n',
        '6,"rs::rs_rank_scatter<y, 2>",FETCH_SIZE,500\n', "7,at::other,FETCH_SIZE,99999\n"])
    write = head + "".join([
        f"1,{cal},WRITE_SIZE,1048576\n", f"2,{cal},WRITE_SIZE,1048576\n",
        "3,rs::rs_tile_histogram<x>,WRITE_SIZE,10\n", "4,rs::rs_tile_histogram<x>,WRITE_SIZE,30\n",
        '5,"void rs::rs_rank_scatter<y, 2>(rs::P<a>, int)",WRITE_SIZE,1000\n',
        '6,"rs::rs_rank_scatter<y, 2>",WRITE_SIZE,1000\n',
        "7,at::other,WRITE_SIZE,5\n"])
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    f.write_text(fetch)
    w.write_text(write)
    out = bench.summarize_pmc("uniform_u32_pairs", str(f), str(w), sorts=2, passes=1, n=1000, command=["x"])
    assert out["calibration"]["fetch_scale"] == 2.0 and out["calibration"]["write_scale"] == 1.0
    hist = out["kernels"]["rs::rs_tile_histogram<x>"]
    assert hist["dispatches"] == 2 and hist["bytes_per_dispatch"] == (2000 * 2 + 20) * 1024
    scat = out["kernels"]["rs::rs_rank_scatter<y, 2>"]
    assert scat["bytes_per_dispatch"] == (500 * 2 + 1000) * 1024
    assert set(out["kernels"]) == {"rs::rs_tile_histogram<x>", "rs::rs_rank_scatter<y, 2>"}
    assert out["bytes_per_sort"] == (2 * hist["bytes_per_dispatch"] + 2 * scat["bytes_per_dispatch"]) // 2
