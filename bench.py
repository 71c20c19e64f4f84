#!/usr/bin/env python3
"""Throughput of the MI355X Recombinant Sort hot path.

Default workload: 268,435,456 uint32 keys uniform over [0, 2^32) with a
uint32 index payload, base-256 digits (4 dimensions), stable ascending sort
through rs_sort_pairs.  One step = one whole sort (per pass: per-tile
counts, scan, stable scatter) with inputs already resident in HBM.

Prints one JSON line: the whole-sort rate in Gkeys/s, the dominant kernel's
(rs_rank_scatter) achieved bandwidth against the 8 TB/s HBM peak, measured
live with HIP events on the launch stream over the timed steps, the CPU
oracle timed on a bounded sample on this host, and the batched form against
one call per array on 4096 arrays of log-uniform size in [2^10, 2^22], and
the served loop (continuous batching vs one launch per request) on a
seeded Poisson trace at equal p99 latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-batched] [--no-served]
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2107_01391_amd", "csrc", f)
                  for f in ("rs_kernels.h", "rs_device.h", "rs_passes.h", "rs_sort.hip", "rs_seg_kernels.h",
                            "rs_str_buckets.h", "rs_segmented.h", "rs_plan.cpp")]
# The other full-size workloads: keys-only decimals over the literal 10^6-cell
# space, fixed-point decimals, and 16-byte strings; algorithmic bytes per key
# are the method's minimum (hash read of the key; scatter read and write of
# key and value; keys only: the key read and written once more).
WORKLOADS = {
    "uniform_decimal_u32": {"kind": "u32", "base": 10, "ndims": 6, "frac": 0, "pairs": False, "alg_bytes": 12,
                            "what": "1,000,000 uint32 keys uniform in [0, 10^6), keys only, base 10, 6 dimensions "
                                    "(literal 10^6-cell space)"},
    "fixed_point_decimals": {"kind": "fixed_i64", "base": 10, "ndims": 9, "frac": 3, "pairs": True,
                             "alg_bytes": 32,
                             "what": "100,000,000 int64 fixed-point decimals (x1000, lognormal, 30% integral, "
                                     "10% repeats), uint32 index payload, base 10, 9 dimensions"},
    "strings16": {"kind": "str", "base": 27, "ndims": 16, "frac": 0, "pairs": True, "alg_bytes": 56,
                  "what": "16,777,216 zero-padded 16-byte lowercase strings, uint32 index payload, base 27, "
                          "16 dimensions"},
}


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_file(name: str) -> str:
    return os.path.join(ROOT, "profiles", f"{name}_pmc.json")


def pmc_summary(n: int, name: str = "uniform_u32_pairs"):
    """The committed PMC summary of a workload, or None when it is missing,
    for another size, or the kernels changed since the counters were taken."""
    try:
        with open(pmc_file(name)) as f:
            pmc = json.load(f)
    except (OSError, ValueError):
        return None
    if pmc.get("kernel_source_sha") != kernel_source_sha() or pmc.get("n") != n:
        return None
    return pmc


def _kernel_bytes(pmc: dict, prefix: str):
    """Scaled HBM bytes per dispatch of the kernels whose name starts with
    `prefix`, summed over those kernels (each a per-dispatch average)."""
    rows = [v for k, v in pmc["kernels"].items() if k.startswith(prefix)]
    return sum(r["bytes_per_dispatch"] for r in rows) if rows else None


def measured_traffic(n: int):
    """HBM bytes per rs_rank_scatter launch (PMC), or None."""
    pmc = pmc_summary(n)
    return _kernel_bytes(pmc, "rs::rs_rank_scatter") if pmc else None


def measured_pass_bytes(n: int):
    """HBM bytes of one whole pass (count, scan, scatter; PMC), or None."""
    pmc = pmc_summary(n)
    if not pmc or not pmc.get("passes"):
        return None
    return pmc["bytes_per_sort"] / pmc["passes"]


def summarize_pmc(name: str, fetch_csv: str, write_csv: str, sorts: int, passes: int | None, n: int,
                  command: list[str]) -> dict:
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch, from two
    rocprofv3 --pmc runs of `bench.py --workload NAME --copy-calibration`),
    scaled by what the same counters read for the calibration copy kernel
    (torch's bitwise_not over 1 GiB: 1 GiB read, 1 GiB written)."""
    import csv
    from collections import defaultdict

    def short(name):
        # "void rs::k<T, ...>(args)" -> "rs::k<T, ...>"
        name = name[5:] if name.startswith("void ") else name
        depth = 0
        for i, c in enumerate(name):
            depth += (c == "<") - (c == ">")
            if c == "(" and depth == 0:
                return name[:i]
        return name

    def read(path, counter):
        per = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                per[short(row["Kernel_Name"])].append(float(row["Counter_Value"]))
        return per

    fetch, write = read(fetch_csv, "FETCH_SIZE"), read(write_csv, "WRITE_SIZE")
    cal_f = [v for k, vs in fetch.items() if "bitwise_not" in k for v in vs]
    cal_w = [v for k, vs in write.items() if "bitwise_not" in k for v in vs]
    gib_kib = float(1 << 20)
    fs = gib_kib / (sum(cal_f) / len(cal_f))
    ws = gib_kib / (sum(cal_w) / len(cal_w))
    kernels = {}
    total = 0.0
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("rs::"):
            continue
        f, w = fetch.get(k, []), write.get(k, [])
        fa = sum(f) / len(f) if f else 0.0
        wa = sum(w) / len(w) if w else 0.0
        b = int(round((fa * fs + wa * ws) * 1024))
        kernels[k] = {"dispatches": max(len(f), len(w)), "FETCH_SIZE_KiB_avg": round(fa, 1),
                      "WRITE_SIZE_KiB_avg": round(wa, 1), "bytes_per_dispatch": b}
        total += b * max(len(f), len(w))
    return {"workload": name, "n": n, "kernel_source_sha": kernel_source_sha(), "commands": command,
            "calibration": {"kernel": "torch bitwise_not over 2^28 int32 (1 GiB read + 1 GiB write)",
                            "fetch_scale": round(fs, 5), "write_scale": round(ws, 5)},
            "sorts": sorts, "passes": passes, "bytes_per_sort": int(round(total / sorts)), "kernels": kernels}


CPU_FULL_FILE = os.path.join(ROOT, "profiles", "cpu_oracle_u32_pairs_268M.json")


def cpu_baseline(w, sample: int) -> dict:
    """The oracle, single-threaded, on the first `sample` pairs.  Its rate
    falls with n (the 2 GiB arrays of the full size miss the host caches
    that a sample's arrays hit), so the full-size time measured once on the
    GPU host (--cpu-full, profiles/cpu_oracle_u32_pairs_268M.json) is
    reported beside it when present."""
    import oracle
    oracle.build(force=False)
    keys, vals = w.keys[:sample], w.vals[:sample]
    t0 = time.perf_counter()
    oracle.sort(keys, vals, kind="u32", base=256, ndims=4, groups=oracle.DEFAULT_GROUPS["uniform_u32_pairs"])
    dt = time.perf_counter() - t0
    out = {"value": round(sample / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "host_cores": os.cpu_count(),
           "kind": "oracle",
           "sample": f"first {sample} pairs of the same seeded input; single-threaded C oracle, gcc -O2, "
                     f"dimension groups [1, 3] (256 buckets, then one 2^24-cell space per bucket); "
                     f"{dt:.1f} s; the rate at the full 2^28 is lower (see full_size)", "seconds": round(dt, 2)}
    try:
        with open(CPU_FULL_FILE) as f:
            full = json.load(f)
        out["full_size"] = {k: full[k] for k in ("n", "seconds", "gkeys_per_s", "host_cores", "host") if k in full}
    except (OSError, ValueError):
        out["full_size"] = None
    return out


def cpu_full(w) -> dict:
    """The oracle once on the whole input (minutes), for the record."""
    import platform

    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.sort(w.keys, w.vals, kind="u32", base=256, ndims=4, groups=oracle.DEFAULT_GROUPS["uniform_u32_pairs"])
    dt = time.perf_counter() - t0
    return {"what": "CPU oracle (single-threaded C, gcc -O2, groups [1, 3]) on the full uniform_u32_pairs input",
            "command": "python bench.py --cpu-full", "n": w.n, "seconds": round(dt, 1),
            "gkeys_per_s": round(w.n / dt / 1e9, 6), "cores": 1, "host_cores": os.cpu_count(),
            "host": platform.processor() or platform.machine()}


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


def oracle_digest_match(keys_out, vals_out, n: int):
    """SHA-256 of the output key and value bytes against the digests the
    oracle wrote for the same seeded workload (tests/golden/digests.json);
    None when none is stored for this size."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "digests.json")) as f:
            rec = json.load(f)["workloads"]["uniform_u32_pairs"]
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("n") != n:
        return None
    hk = hashlib.sha256(keys_out[: 4 * n].cpu().numpy().data).hexdigest()
    hv = hashlib.sha256(vals_out[: 4 * n].cpu().numpy().data).hexdigest()
    return hk == rec["keys_sha256"] and hv == rec["vals_sha256"]


def calibration_copy(torch) -> None:
    """A plain streaming kernel of known size for the PMC byte counters:
    reads 1 GiB and writes 1 GiB (torch's elementwise bitwise_not)."""
    a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(2):
        torch.bitwise_not(a, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


PROF_KERNELS = ("rs_tile_histogram", "rs_cell_scan", "rs_rank_scatter", "rs_digit_hash_histogram", "rs_fill",
                "rs_cell_count", "rs_cell_emit", "rs_small_sort", "rs_copy", "rs_str_bucket_count",
                "rs_str_bucket_sort", "rs_seg_plan", "rs_seg_tiles")


def run_workload(torch, B, api, workloads, name: str, steps: int, warmup: int) -> dict:
    """One of WORKLOADS at full size through rs_sort_pairs / rs_sort_keys
    with the default tuning: median whole-sort time over `steps` event-timed
    sorts, per-kernel time (HIP events on the launch stream), the output's
    SHA-256 against the oracle's digest, and the whole sort's share of the
    HBM peak from the algorithmic bytes and from the committed counters."""
    spec = WORKLOADS[name]
    print(f"[bench] {name}: generating", file=sys.stderr, flush=True)
    w = getattr(workloads, name)()
    n = w.n
    d = B.key_desc(spec["kind"], base=spec["base"], ndims=spec["ndims"], frac_digits=spec["frac"])
    keys = api.to_device(w.keys)
    vals = api.to_device(w.vals) if spec["pairs"] else None
    del w
    ko = torch.empty_like(keys)
    vo = torch.empty_like(vals) if vals is not None else None
    tmp = api.empty_device(B.rs_temp_bytes(d, n, spec["pairs"]))
    stream = torch.cuda.current_stream()

    def once():
        if spec["pairs"]:
            B.rs_sort_pairs(d, keys, ko, vals, vo, n, tmp, tmp.numel(), stream)
        else:
            B.rs_sort_keys(d, keys, ko, n, tmp, tmp.numel(), stream)

    for _ in range(warmup):
        once()
    torch.cuda.synchronize()
    evs = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        once()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    # per-kernel times from the same number of sorts again, each launch
    # timed by HIP events (kept out of the sort times above)
    B.rs_prof_enable(True)
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    kern = {}
    for k in PROF_KERNELS:
        c, ms_k = B.rs_prof_query(k)
        if c:
            kern[k] = {"launches_per_sort": c // steps, "ms_per_sort": round(ms_k / steps, 4)}
    B.rs_prof_enable(False)
    times = sorted(a.elapsed_time(b) for a, b in evs)
    ms = times[len(times) // 2]
    digest = None
    try:
        with open(os.path.join(ROOT, "tests", "golden", "digests.json")) as f:
            rec = json.load(f)["workloads"][name]
        if rec.get("n") == n:
            kb = keys.numel()
            digest = hashlib.sha256(ko[:kb].cpu().numpy().data).hexdigest() == rec["keys_sha256"]
            if vo is not None:
                digest = digest and hashlib.sha256(vo[: 4 * n].cpu().numpy().data).hexdigest() == rec["vals_sha256"]
    except (OSError, ValueError, KeyError):
        pass
    alg = spec["alg_bytes"] * n
    line = {"workload": name, "what": spec["what"], "n": n, "ms": round(ms, 4), "ms_min": round(times[0], 4),
            "gkeys_per_s": round(n / (ms / 1e3) / 1e9, 3), "algorithmic_bytes_per_key": spec["alg_bytes"],
            "algorithmic_frac_of_peak": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_ms_per_sort": kern, "oracle_digest_match": digest}
    pmc = pmc_summary(n, name)
    line["measured_bytes_per_sort"] = pmc["bytes_per_sort"] if pmc else None
    line["measured_frac_of_peak"] = (round(pmc["bytes_per_sort"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                     if pmc else None)
    del keys, vals, ko, vo, tmp
    torch.cuda.empty_cache()
    return line


def graph_tuned_batched(torch, B, desc, keys, keys_out, vals, vals_out, off_dev, count: int, total: int,
                        offsets) -> dict:
    """The batched form as the workload states it: the autotuner picks the
    pass width and tile shape on these arrays (rs_tune_batched), the
    sequence is captured once as a HIP graph (rs_graph_sort_batched) and
    replayed; replays are event-timed and their output spot-checked."""
    st = torch.cuda.current_stream()
    tt = torch.empty(B.rs_tune_temp_bytes(desc, total, count, True), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    best, best_ms = B.rs_tune_batched(desc, keys, keys_out, vals, vals_out, off_dev, count, total, tt, tt.numel(),
                                      st, reps=2)
    tune_s = time.perf_counter() - t0
    del tt
    torch.cuda.empty_cache()
    tmp = torch.empty(B.rs_batched_temp_bytes(desc, total, count, True), dtype=torch.uint8, device="cuda")
    g = B.rs_graph_sort_batched(desc, keys, keys_out, vals, vals_out, off_dev, count, total, tmp, tmp.numel())
    g.launch(st)
    torch.cuda.synchronize()
    reps = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        g.launch(st)
        b.record(st)
        b.synchronize()
        reps.append(a.elapsed_time(b))
    good = True
    for i in (0, count // 3, count - 1):
        lo, hi = int(offsets[i]), int(offsets[i + 1])
        k = keys_out[lo:hi].to(torch.int64) & 0xFFFFFFFF
        v = vals_out[lo:hi].to(torch.int64)
        src = keys[lo:hi].to(torch.int64) & 0xFFFFFFFF
        good = good and bool((k[1:] >= k[:-1]).all()) and bool((src[v] == k).all())
        good = good and bool(((k[1:] != k[:-1]) | (v[1:] > v[:-1])).all())
    g.close()
    del tmp
    torch.cuda.empty_cache()
    ms = min(reps)
    return {"makespan_ms": round(ms, 3), "p50_ms": round(ms, 3), "p99_ms": round(ms, 3),
            "gkeys_per_s": round(total / (ms / 1e3) / 1e9, 3), "replays_ms": [round(r, 3) for r in reps],
            "tuned": best.as_dict(), "tuner_best_ms": round(best_ms, 3), "tuning_seconds": round(tune_s, 2),
            "spot_check": good}


def batched_vs_per_array(torch, B, workloads, count: int) -> dict:
    """`count` arrays with log-uniform sizes in [2^10, 2^22] (the seeded size
    law), uniform u32 keys and local-index payloads drawn on the device.
    Per-array: one rs_sort_pairs call per array, on 1 and on 4 streams (the
    better is kept); an array's latency runs from the common start to the
    event after its own sort.  Batched: one rs_sort_batched sequence, in
    which every array completes at the makespan, eagerly with the default
    tuning, and as the workload states it (graph_tuned): tuned, captured
    once in a HIP graph, replayed."""
    from paper_2107_01391_amd import api
    sizes = workloads.batched_sizes(count)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    g = torch.Generator(device="cuda")
    g.manual_seed(workloads.SEED_BASE + 4)
    keys = torch.randint(0, 2**32, (total,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
    starts = torch.repeat_interleave(torch.from_numpy(offsets[:-1].astype(np.int64)).cuda(),
                                     torch.from_numpy(sizes).cuda())
    vals = (torch.arange(total, dtype=torch.int64, device="cuda") - starts).to(torch.int32)
    del starts
    keys_out, vals_out = torch.empty_like(keys), torch.empty_like(vals)
    desc = B.key_desc("u32", base=256, ndims=4)
    off_dev = api.to_device(offsets)
    res = {"arrays": count, "total_pairs": total, "size_law": "log-uniform [2^10, 2^22], seeded",
           "keys": "uniform u32 drawn on the device (torch Philox, seeded); local-index payload"}

    def run(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            r = fn()
            if best is None or r["makespan_ms"] < best["makespan_ms"]:
                best = r
        return best

    # batched: one sequence for every array
    tmp = torch.empty(B.rs_batched_temp_bytes(desc, total, count, True), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()

    def batched_once():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        B.rs_sort_batched(desc, keys, keys_out, vals, vals_out, off_dev, count, total, tmp, tmp.numel(), st)
        b.record(st)
        b.synchronize()
        ms = a.elapsed_time(b)
        return {"makespan_ms": round(ms, 3), "p50_ms": round(ms, 3), "p99_ms": round(ms, 3)}

    res["batched"] = run(batched_once)
    # spot check: three arrays sorted with ties in input order
    for i in (0, count // 2, count - 1):
        lo, hi = int(offsets[i]), int(offsets[i + 1])
        k = keys_out[lo:hi].to(torch.int64) & 0xFFFFFFFF
        v = vals_out[lo:hi].to(torch.int64)
        src = keys[lo:hi].to(torch.int64) & 0xFFFFFFFF
        good = bool((k[1:] >= k[:-1]).all()) and bool((src[v] == k).all())
        good = good and bool(((k[1:] != k[:-1]) | (v[1:] > v[:-1])).all())
        res.setdefault("spot_check", True)
        res["spot_check"] = res["spot_check"] and good
    del tmp
    torch.cuda.empty_cache()
    res["graph_tuned"] = graph_tuned_batched(torch, B, desc, keys, keys_out, vals, vals_out, off_dev, count, total,
                                             offsets)
    B.rs_tuning_clear()

    per = []
    for nstreams in (1, 4):
        streams = [torch.cuda.Stream() for _ in range(nstreams)]
        tmps = [torch.empty(B.rs_temp_bytes(desc, int(sizes.max()), True), dtype=torch.uint8, device="cuda")
                for _ in range(nstreams)]

        def per_array_once():
            start = torch.cuda.Event(enable_timing=True)
            start.record(st)
            for s in streams:
                s.wait_event(start)
            done = []
            for i in range(count):
                s = streams[i % nstreams]
                lo, hi = int(offsets[i]), int(offsets[i + 1])
                B.rs_sort_pairs(desc, keys[lo:], keys_out[lo:], vals[lo:], vals_out[lo:], hi - lo,
                                tmps[i % nstreams], tmps[i % nstreams].numel(), s)
                e = torch.cuda.Event(enable_timing=True)
                e.record(s)
                done.append(e)
            torch.cuda.synchronize()
            lat = np.array([start.elapsed_time(e) for e in done])
            return {"makespan_ms": round(float(lat.max()), 3), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3), "streams": nstreams}

        per.append(run(per_array_once))
        del tmps
    res["per_array"] = min(per, key=lambda r: r["makespan_ms"])
    res["per_array_all"] = per
    for k in ("batched", "per_array"):
        res[k]["gkeys_per_s"] = round(total / (res[k]["makespan_ms"] / 1e3) / 1e9, 3)
    res["batched_speedup"] = round(res["per_array"]["makespan_ms"] / res["batched"]["makespan_ms"], 3)
    res["graph_tuned_speedup"] = round(res["per_array"]["makespan_ms"] / res["graph_tuned"]["makespan_ms"], 3)
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=FULL_N)
    ap.add_argument("--cpu-sample", type=int, default=1 << 25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-arrays", type=int, default=4096)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=10000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write kernel (scale reference for PMC byte counters)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS),
                    help="time only this workload (default tuning) and print its line")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other full-size workloads")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph replay of the sort")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the CPU oracle on the full 2^28-pair input (minutes) and record it under profiles/")
    ap.add_argument("--pmc-summary", metavar="WORKLOAD",
                    help="write profiles/WORKLOAD_pmc.json from the --fetch and --write counter CSVs")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sorts", type=int, help="sorts in the profiled run (warm-up + timed)")
    ap.add_argument("--passes", type=int, help="passes of one sort in the profiled run")
    ap.add_argument("--command", action="append", default=[], help="profiling command, for the record")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sort runs on a single MI355X. Several GPUs would split the "
              "count space by the leading digit group and exchange pairs with one all-to-all; that is not "
              "implemented, so only --gpus 1 runs", file=sys.stderr)
        return 2

    if args.pmc_summary:
        from paper_2107_01391_amd import workloads as wl
        n = args.n if args.pmc_summary == "uniform_u32_pairs" else wl.FULL_SIZES[getattr(
            wl, args.pmc_summary.upper())]
        out = summarize_pmc(args.pmc_summary, args.fetch, args.write, args.sorts, args.passes, n, args.command)
        with open(pmc_file(args.pmc_summary), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps({k: out[k] for k in ("workload", "n", "sorts", "bytes_per_sort")}))
        return 0

    if args.cpu_full:
        from paper_2107_01391_amd import workloads as wl
        rec = cpu_full(wl.uniform_u32_pairs(FULL_N))
        with open(CPU_FULL_FILE, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return 0

    import torch

    from paper_2107_01391_amd import _binding as B
    from paper_2107_01391_amd import api, workloads

    if args.copy_calibration:
        calibration_copy(torch)
    if args.workload:
        print(json.dumps(run_workload(torch, B, api, workloads, args.workload, args.steps, args.warmup)), flush=True)
        return 0

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

    def step():
        B.rs_sort_pairs(desc, keys, keys_out, vals, vals_out, n, tmp, tmp.numel(), stream)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ok = check_sorted(torch, keys, keys_out, vals_out, n)
    print(f"[bench] output check {'ok' if ok else 'FAILED'}; timing {args.steps} steps", file=sys.stderr, flush=True)

    # the timed steps: the sorts alone (the per-kernel event pairs below add
    # a marker before and after every launch, about 1.7% of the sort)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same number of steps again with every kernel launch timed by HIP
    # events on its stream: the per-kernel figures of the roofline
    print(f"[bench] per-kernel timing over {args.steps} more steps", file=sys.stderr, flush=True)
    B.rs_prof_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    launches, total_ms = B.rs_prof_query("rs_rank_scatter")
    kernel_ms = {k: round(B.rs_prof_query(k)[1] / args.steps, 4)
                 for k in ("rs_tile_histogram", "rs_cell_scan", "rs_rank_scatter", "rs_digit_hash_histogram")}
    B.rs_prof_enable(False)

    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    wall_ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e9
    avg_ms = total_ms / max(launches, 1)
    per_launch_bytes = n * 16  # read key + value, write key + value (4 B each)
    achieved = per_launch_bytes / (avg_ms / 1e3) / 1e9
    traffic = measured_traffic(n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "rs_rank_scatter", "launches": launches, "avg_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": per_launch_bytes}
    passes = launches // max(args.steps, 1)
    planned = passes * 20  # per pass: count read 4 B, scatter read 8 B and write 8 B
    whole = {"algorithmic_bytes_per_pair": 20, "planned_bytes_per_pair": planned, "passes": passes,
             "algorithmic_GBps": round(20 * n / (ms_per_step / 1e3) / 1e9, 1),
             "planned_GBps": round(planned * n / (ms_per_step / 1e3) / 1e9, 1),
             "planned_frac_of_peak": round(planned * n / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
             "wall_ms_per_step": round(wall_ms_per_step, 4), "kernel_ms_per_step": kernel_ms}
    pass_bytes = measured_pass_bytes(n)
    # counter-measured bytes of every kernel of the sort over its time: the
    # whole sort's share of the HBM peak (null when the counters are stale)
    whole["measured_bytes_per_step"] = pass_bytes * passes if pass_bytes else None
    whole["measured_frac_of_peak"] = (round(pass_bytes * passes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                      if pass_bytes else None)
    # the timed steps' output, byte for byte, against the oracle's digest
    digest_ok = oracle_digest_match(keys_out, vals_out, n)
    print(f"[bench] oracle digest {'match' if digest_ok else ('MISMATCH' if digest_ok is False else 'not stored')}",
          file=sys.stderr, flush=True)

    # the same sort captured once as a HIP graph (rs_graph_sort) and replayed
    # the same number of steps: the same kernels on the same data, fewer
    # gaps between dependent launches; reported beside the plain call
    graph = None
    if not args.no_graph:
        keys_out.zero_()
        vals_out.zero_()
        g = B.rs_graph_sort(desc, keys, keys_out, vals, vals_out, n, tmp, tmp.numel())
        for _ in range(args.warmup):
            g.launch(stream)
        torch.cuda.synchronize()
        g_ok = oracle_digest_match(keys_out, vals_out, n)
        ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ga.record(stream)
        for _ in range(args.steps):
            g.launch(stream)
        gb.record(stream)
        torch.cuda.synchronize()
        g_ms = ga.elapsed_time(gb) / args.steps
        g.close()
        graph = {"ms_per_step": round(g_ms, 4), "gkeys_per_s": round(n / (g_ms / 1e3) / 1e9, 3),
                 "oracle_digest_match": g_ok}
    del keys_out, vals_out, tmp
    torch.cuda.empty_cache()

    others = None
    if not args.no_workloads:
        others = [run_workload(torch, B, api, workloads, name, 10, 2)
                  for name in ("uniform_decimal_u32", "fixed_point_decimals", "strings16")]

    batched = None
    if not args.no_batched:
        print("[bench] batched vs per-array", file=sys.stderr, flush=True)
        batched = batched_vs_per_array(torch, B, workloads, args.batched_arrays)
        torch.cuda.empty_cache()

    served = None
    if not args.no_served:
        from paper_2107_01391_amd import serve
        print("[bench] served: per-request vs batched", file=sys.stderr, flush=True)
        # p99 is the 1%-tail of the latencies: 10,000 requests per rate put
        # 100 of them past it (the 3-seed study with 20,000 per rate is in
        # profiles/served_u32_pairs_loguniform_sweep.md)
        rows = serve.sweep([2000.0, 2500.0, 3000.0, 4000.0, 8000.0, 16000.0, 0.0], args.served_requests, 1000,
                           1 << 28, 4, verbose=False)
        gate = serve.gate(rows)
        served = {"trace": f"{args.served_requests} requests after 1000 warm-up, sizes log-uniform [2^10, 2^22], "
                           "Poisson arrivals (rate 0 = closed loop), arena 2^28 keys, 4 streams",
                  "rows": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()} for r in rows],
                  "equal_p99": gate, "crossover": serve.crossover(gate)}

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
                   "n": n, "passes": passes},
        "roofline": roofline, "whole_sort": whole, "graph_replay": graph, "cpu_baseline": cpu, "workloads": others,
        "batched_vs_per_array": batched,
        "served": served, "output_check": ok, "oracle_digest_match": digest_ok,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
