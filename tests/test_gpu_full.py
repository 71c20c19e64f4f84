"""Full-size parity: every workload at its full size, in the launch
configuration the benchmark times (default tuning), compared byte for byte
with the CPU oracle through the SHA-256 digests that
tests/golden/make_digests.py wrote by calling only the oracle."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "digests.json")) as f:
    DIGESTS = json.load(f)["workloads"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data).hexdigest()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    B.rs_tuning_clear()


def _single(name, maker, kind, base, ndims, frac=0, pairs=True):
    import torch
    rec = DIGESTS[name]
    w = maker()
    n = w.n
    assert n == rec["n"]
    _say(f"full {name}: n={n}")
    d = B.key_desc(kind, base=base, ndims=ndims, frac_digits=frac)
    kd = api.to_device(w.keys)
    ko = torch.empty_like(kd)
    tmp = api.empty_device(B.rs_temp_bytes(d, n, pairs))
    if pairs:
        vd = api.to_device(w.vals)
        vo = torch.empty_like(vd)
        B.rs_sort_pairs(d, kd, ko, vd, vo, n, tmp, tmp.numel())
    else:
        B.rs_sort_keys(d, kd, ko, n, tmp, tmp.numel())
    torch.cuda.synchronize()
    del tmp, kd
    gk = ko.cpu().numpy()
    assert sha(gk) == rec["keys_sha256"], f"{name}: keys differ from the oracle"
    if pairs:
        assert sha(vo.cpu().numpy()) == rec["vals_sha256"], f"{name}: values differ from the oracle"


def test_full_uniform_decimal_keys_literal():
    """10^6 keys over a 10^6-cell space, keys only: the literal form."""
    _single("uniform_decimal_u32", workloads.uniform_decimal_u32, "u32", 10, 6, pairs=False)


def test_full_u32_pairs_268M():
    """The benchmark's workload: 2^28 uint32 pairs, base 256."""
    _single("uniform_u32_pairs", workloads.uniform_u32_pairs, "u32", 256, 4)


def test_full_fixed_point_100M():
    """10^8 int64 fixed-point decimals (skewed lognormal, duplicates)."""
    _single("fixed_point_decimals", workloads.fixed_point_decimals, "fixed_i64", 10, 9, frac=3)


def test_full_strings_16M():
    """2^24 zero-padded 16-byte lowercase strings."""
    _single("strings16", workloads.strings16, "str", 27, 16)


def test_full_batched_4096_arrays():
    """4096 arrays, log-uniform sizes in [2^10, 2^22], one rs_sort_batched
    sequence; digest = SHA-256 of the per-array digests in order."""
    import torch
    rec = DIGESTS["batched_u32"]
    _say("full batched: generating")
    keys, vals, offs = workloads.batched_u32()
    total, nseg = int(offs[-1]), offs.shape[0] - 1
    assert total == rec["n"] and nseg == rec["arrays"]
    d = B.key_desc("u32", base=256, ndims=4)
    kd = api.to_device(keys)
    vd = api.to_device(vals)
    del keys, vals
    od = api.to_device(offs)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, total, nseg, True))
    _say(f"full batched: sorting {total} pairs in {nseg} arrays")
    B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    del tmp, kd, vd
    gk = ko.cpu().numpy().view(np.uint32)
    gv = vo.cpu().numpy().view(np.uint32)
    _say("full batched: hashing")
    hk, hv = hashlib.sha256(), hashlib.sha256()
    for i in range(nseg):
        a, b = int(offs[i]), int(offs[i + 1])
        dk, dv = sha(gk[a:b]), sha(gv[a:b])
        if i < len(rec["first_arrays"]):
            size, ek, ev = rec["first_arrays"][i]
            assert size == b - a
            assert dk == ek and dv == ev, f"array {i} ({b - a} keys) differs from the oracle"
        hk.update(dk.encode())
        hv.update(dv.encode())
    assert hk.hexdigest() == rec["keys_sha256"] and hv.hexdigest() == rec["vals_sha256"]
