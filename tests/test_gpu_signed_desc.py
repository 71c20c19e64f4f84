"""Signed keys and descending order on the GPU against the oracle (both
beyond the paper, which sorts non-negative keys ascending): element by
element, through every pass form (chained, prescanned, batched), pairs and
keys only, in place."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads
from tests.gpu_helpers import assert_same, fast_groups, gpu_sort, oracle_sort

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()


@pytest.fixture(params=["chained", "prescanned"])
def form(request, monkeypatch):
    monkeypatch.setenv("RS_PRESCAN_MIN_N", str(1 << 40) if request.param == "chained" else "1")
    yield request.param


def _signed(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "i32":
        lo, hi = -2**31, 2**31 - 1
        k = rng.integers(lo, hi, n, dtype=np.int64, endpoint=True).astype(np.int32)
    else:
        lo, hi = -2**63, 2**63 - 1
        k = rng.integers(lo, hi, n, dtype=np.int64, endpoint=True)
    k[::9] = lo  # the extremes of the type
    k[1::13] = hi
    if n > 3:
        k[2::5] = k[3]  # duplicates: ties keep input order
    return k


@pytest.mark.parametrize("kind,base,ndims", [("i32", 256, 4), ("i32", 10, 10), ("i64", 256, 8), ("i64", 16, 16)])
@pytest.mark.parametrize("n", [1, 4097, 100_003])
def test_signed_pairs(form, kind, base, ndims, n):
    _say(f"signed {kind} base {base} n={n} {form}")
    keys = _signed(kind, n, n + base)
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, kind, base, ndims)
    ok, ov = oracle_sort(keys, vals, kind, base, ndims)
    assert_same(gk, gv, ok, ov)
    assert np.array_equal(ok, np.sort(keys, kind="stable"))  # and the integers' own order


@pytest.mark.parametrize("kind", ["i32", "i64"])
def test_signed_keys_only_descending_in_place(form, kind):
    _say(f"signed {kind} keys only, descending, in place, {form}")
    keys = _signed(kind, 77_777, 3)
    ndims = 4 if kind == "i32" else 8
    gk, _ = gpu_sort(keys, None, kind, 256, ndims, descending=True)
    ok, _ = oracle_sort(keys, None, kind, 256, ndims, descending=True)
    assert_same(gk, None, ok, None)
    vals = np.arange(keys.shape[0], dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, kind, 256, ndims, descending=True, in_place=True)
    ok, ov = oracle_sort(keys, vals, kind, 256, ndims, descending=True)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("case", ["u32", "u64", "fixed", "str", "base10"])
def test_descending_pairs(form, case):
    _say(f"descending {case} {form}")
    if case == "u32":
        w = workloads.uniform_u32_pairs(150_001)
        args = ("u32", 256, 4)
        keys, vals = w.keys, w.vals
        keys[::7] = keys[5]
    elif case == "u64":
        rng = np.random.default_rng(4)
        keys = rng.integers(0, 2**64, 60_001, dtype=np.uint64)
        vals = np.arange(keys.shape[0], dtype=np.uint32)
        args = ("u64", 256, 8)
    elif case == "fixed":
        w = workloads.fixed_point_decimals(120_007)
        keys, vals = w.keys, w.vals
        args = ("fixed_i64", 10, 9)
    elif case == "str":
        w = workloads.strings16(40_001)
        keys, vals = w.keys, w.vals
        args = ("str", 27, 16)
    else:
        w = workloads.uniform_decimal_u32(90_001)
        keys, vals = w.keys, np.arange(90_001, dtype=np.uint32)
        args = ("u32", 10, 6)
    gk, gv = gpu_sort(keys, vals, *args, descending=True)
    ok, ov = oracle_sort(keys, vals, *args, descending=True)
    assert_same(gk, gv, ok, ov)


def test_descending_decimal_keys_only_not_literal():
    """Keys only on a small space would take the literal (ascending) form;
    descending must not."""
    _say("descending decimal keys only")
    w = workloads.uniform_decimal_u32(50_000)
    gk, _ = gpu_sort(w.keys, None, "u32", 10, 6, descending=True)
    ok, _ = oracle_sort(w.keys, None, "u32", 10, 6, descending=True)
    assert_same(gk, None, ok, None)


@pytest.mark.parametrize("kind", ["u32", "i32"])
def test_batched_descending_and_signed(kind):
    import torch
    _say(f"batched {kind} descending")
    keys, vals, offs = workloads.batched_u32(count=30, lo=10, hi=60_000)
    if kind == "i32":
        keys = keys.view(np.int32).copy()
    total, nseg = int(offs[-1]), offs.shape[0] - 1
    d = B.key_desc(kind, base=256, ndims=4, descending=True)
    kd, vd, od = api.to_device(keys), api.to_device(vals), api.to_device(offs)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, total, nseg, True))
    B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind=kind, base=256, ndims=4,
                                     groups=fast_groups(kind, 256, 4), descending=True)
    dt = np.uint32 if kind == "u32" else np.int32
    assert np.array_equal(api.to_host(ko, dt, (total,)), ok)
    assert np.array_equal(api.to_host(vo, np.uint32, (total,)), ov)


def _byte_rows(n, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    rows[:, 3:] = np.where(rng.random((n, 13)) < 0.3, 0, rows[:, 3:])  # padding-like zeros
    if n > 2:
        rows[::7] = rows[2]  # duplicates
    return rows


@pytest.mark.parametrize("desc", [False, True])
@pytest.mark.parametrize("n", [1, 2049, 70_001])
def test_byte_strings(form, desc, n):
    """16-byte keys over every byte value (base 256): memcmp order."""
    _say(f"byte strings n={n} desc={desc} {form}")
    keys = _byte_rows(n, n)
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "str", 256, 16, descending=desc)
    ok, ov = oracle_sort(keys, vals, "str", 256, 16, descending=desc)
    assert_same(gk, gv, ok, ov)
    if n > 1:
        rows = [bytes(r) for r in keys]
        assert [bytes(r) for r in gk] == sorted(rows, reverse=desc)


def test_byte_strings_batched_keys_only():
    import torch
    _say("byte strings batched keys only")
    keys = _byte_rows(30_000, 5)
    offs = np.array([0, 1, 2000, 2049, 10_000, 30_000], np.uint64)
    d = B.key_desc("str", base=256, ndims=16)
    kd, od = api.to_device(keys), api.to_device(offs)
    ko = torch.empty_like(kd)
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, 30_000, 5, False))
    B.rs_sort_batched(d, kd, ko, None, None, od, 5, 30_000, tmp, tmp.numel())
    torch.cuda.synchronize()
    got = api.to_host(ko, np.uint8, (30_000, 16))
    for a, b in zip(offs[:-1], offs[1:]):
        want = sorted(bytes(r) for r in keys[int(a):int(b)])
        assert [bytes(r) for r in got[int(a):int(b)]] == want
