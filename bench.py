#!/usr/bin/env python3
"""Throughput of the MI355X Recombinant Sort hot path.

Default workload: 268,435,456 uint32 keys uniform over [0, 2^32) with a
uint32 index payload, base-256 digits (4 dimensions), stable ascending sort
through rs_sort_pairs.  One step = one whole sort (histogram, scans and the
four stable passes) with inputs already resident in HBM.

Prints one JSON line: the whole-sort rate in Gkeys/s, the dominant kernel's
(rs_rank_scatter) achieved bandwidth against the 8 TB/s HBM peak, measured
live with HIP events on the launch stream over the timed steps, and the CPU
oracle timed on a bounded sample on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Gkeys/s + % HBM peak, 256M u32 KV sort; batched vs per-array at p99 latency"
HBM_PEAK_GBS = 8000.0
FULL_N = 1 << 28
PMC_FILE = os.path.join(ROOT, "profiles", "rank_scatter_u32_pairs_268M_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2107_01391_amd", "csrc", f) for f in ("rs_kernels.h", "rs_device.h")]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n: int):
    """HBM bytes per rs_rank_scatter launch from the committed PMC summary,
    or None when it is missing, for another size, or the kernel changed."""
    try:
        with open(PMC_FILE) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_source_sha") != kernel_source_sha() or pmc.get("n") != n:
        return None
    return pmc.get("hbm_bytes_per_launch")


def cpu_baseline(w, sample: int) -> dict:
    import oracle
    oracle.build(force=False)
    keys, vals = w.keys[:sample], w.vals[:sample]
    t0 = time.perf_counter()
    oracle.sort(keys, vals, kind="u32", base=256, ndims=4, groups=oracle.DEFAULT_GROUPS["uniform_u32_pairs"])
    dt = time.perf_counter() - t0
    return {"value": round(sample / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample} pairs of the same seeded input; single-threaded C oracle, gcc -O2, "
                      f"dimension groups [1, 3] (256 buckets, then one 2^24-cell space per bucket); "
                      f"{dt:.1f} s", "seconds": round(dt, 2)}


def check_sorted(torch, keys_in, keys_out, vals_out, n):
    """Sanity check on the device: keys non-decreasing, ties in input order,
    and keys_out[i] == keys_in[vals_out[i]]."""
    ki = keys_in[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    ko = keys_out[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    vo = vals_out[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    ok = bool((ko[1:] >= ko[:-1]).all()) and bool(((ko[1:] != ko[:-1]) | (vo[1:] > vo[:-1])).all())
    ok = ok and bool((ki[vo] == ko).all())
    del ki, ko, vo
    return ok


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=FULL_N)
    ap.add_argument("--cpu-sample", type=int, default=1 << 26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (scale reference for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sort runs on a single MI355X; a run on more GPUs is not part "
              "of this build (see the sharding notes in DESIGN.md)", file=sys.stderr)
        return 2

    import torch

    from paper_2107_01391_amd import _binding as B
    from paper_2107_01391_amd import api, workloads

    n = args.n
    print(f"[bench] generating {n} pairs", file=sys.stderr, flush=True)
    w = workloads.uniform_u32_pairs(n)
    keys = api.to_device(w.keys)
    vals = api.to_device(w.vals)
    keys_out = api.empty_device(keys.numel())
    vals_out = api.empty_device(vals.numel())
    desc = B.key_desc("u32", base=256, ndims=4)
    need = B.rs_temp_bytes(desc, n, True)
    tmp = api.empty_device(need)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        B.rs_sort_pairs(desc, keys, keys_out, vals, vals_out, n, tmp, tmp.numel(), stream)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ok = check_sorted(torch, keys, keys_out, vals_out, n)
    print(f"[bench] output check {'ok' if ok else 'FAILED'}; timing {args.steps} steps", file=sys.stderr, flush=True)

    B.rs_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, total_ms = B.rs_prof_query("rs_rank_scatter")
    hist_launches, hist_ms = B.rs_prof_query("rs_digit_hash_histogram")
    B.rs_prof_enable(False)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e9
    avg_ms = total_ms / max(launches, 1)
    per_launch_bytes = n * 16  # read key + value, write key + value (4 B each)
    achieved = per_launch_bytes / (avg_ms / 1e3) / 1e9
    traffic = measured_traffic(n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "rs_rank_scatter", "launches": launches, "avg_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": per_launch_bytes}
    whole = {"algorithmic_bytes_per_pair": 20, "planned_bytes_per_pair": 68,
             "algorithmic_GBps": round(20 * n / (ms_per_step / 1e3) / 1e9, 1),
             "planned_GBps": round(68 * n / (ms_per_step / 1e3) / 1e9, 1),
             "histogram_avg_ms": round(hist_ms / max(hist_launches, 1), 4)}

    cpu = None
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        print(f"[bench] cpu oracle on {sample} pairs", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, sample)

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"uniform_u32_pairs: {n} uint32 keys uniform over [0, 2^32), uint32 index payload, "
                               "base 256, 4 dimensions, stable ascending (rs_sort_pairs)",
                   "n": n, "passes": 4, "tile_keys": 4096},
        "roofline": roofline, "whole_sort": whole, "cpu_baseline": cpu, "output_check": ok,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
