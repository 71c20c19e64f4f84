"""Writes tests/golden/digests.json: SHA-256 of the CPU oracle's output on
every full-size workload (the GPU tests compare their output bytes with
these).  Calls only the oracle and the seeded generators.

    python -m tests.golden.make_digests [workload ...]

Workloads: uniform_decimal_u32 uniform_u32_pairs fixed_point_decimals
strings16 batched_u32.  Each uses the oracle's default dimension groups for
that workload.  Takes minutes for the large ones; the batched workload's
arrays are sorted by DIGEST_WORKERS processes (default 6) and its digest is
the SHA-256 of the per-array digests (hex, in array order).
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

import oracle
from paper_2107_01391_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "digests.json")

SPECS = {
    "uniform_decimal_u32": ("u32", 10, 6),
    "uniform_u32_pairs": ("u32", 256, 4),
    "fixed_point_decimals": ("fixed_i64", 10, 9),
    "strings16": ("str", 27, 16),
    "batched_u32": ("u32", 256, 4),
}
MAKERS = {
    "uniform_decimal_u32": workloads.uniform_decimal_u32,
    "uniform_u32_pairs": workloads.uniform_u32_pairs,
    "fixed_point_decimals": workloads.fixed_point_decimals,
    "strings16": workloads.strings16,
}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data).hexdigest()


WORKERS = int(os.environ.get("DIGEST_WORKERS", "6"))


def _batched_one(job):
    i, size, kind, base, ndims, groups = job
    keys, vals = workloads.batched_array(i, size)
    ko, vo, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups)
    return sha(ko), sha(vo)


def one(name: str) -> dict:
    kind, base, ndims = SPECS[name]
    groups = oracle.DEFAULT_GROUPS[name]
    t0 = time.perf_counter()
    if name == "batched_u32":
        # arrays are independent: sort them in worker processes; the digest of
        # the whole batch is the SHA-256 of the per-array digests in order
        sizes = workloads.batched_sizes()
        hk, hv = hashlib.sha256(), hashlib.sha256()
        per = []
        jobs = [(i, int(s), kind, base, ndims, groups) for i, s in enumerate(sizes)]
        with mp.get_context("fork").Pool(WORKERS) as pool:
            for i, (dk, dv) in enumerate(pool.imap(_batched_one, jobs, chunksize=4)):
                hk.update(dk.encode())
                hv.update(dv.encode())
                if i < 64:
                    per.append([int(sizes[i]), dk, dv])
        rec = {"n": int(sizes.sum()), "arrays": int(sizes.shape[0]), "digest_of_array_digests": True,
               "keys_sha256": hk.hexdigest(), "vals_sha256": hv.hexdigest(), "first_arrays": per}
    else:
        w = MAKERS[name]()
        ko, vo, st = oracle.sort(w.keys, w.vals, kind=kind, base=base, ndims=ndims, groups=groups)
        rec = {"n": w.n, "keys_sha256": sha(ko), "vals_sha256": None if vo is None else sha(vo),
               "cells_visited": st.cells_visited}
    rec.update({"kind": kind, "base": base, "ndims": ndims, "groups": groups,
                "oracle_seconds": round(time.perf_counter() - t0, 1)})
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["numpy_version"] = workloads.numpy_version()
    data["note"] = "SHA-256 of the oracle's output bytes (keys, then uint32 values) per full-size workload"
    for name in names:
        print(f"{name} ...", flush=True)
        data.setdefault("workloads", {})[name] = one(name)
        print(json.dumps(data["workloads"][name])[:300], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(SPECS))
