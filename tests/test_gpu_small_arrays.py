"""Arrays of up to 4096 keys, sorted whole on chip.  In the batched form:
rs_local_sort (4-bit sub-passes over each cell index, for plans of two or
more passes) and rs_small_sort (one pass, ballot ranking).  A single short
array given to rs_sort_pairs / rs_sort_keys: one workgroup of rs_local_sort.
Every array is compared with the oracle's sort of that array alone, at every
length class a tile meets: empty, single, one short of / exactly / one past
a 16-key run, ragged, and the 4096-key maximum."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads
from tests.gpu_helpers import assert_same, fast_groups, gpu_sort, key_dtype, key_shape

pytestmark = pytest.mark.gpu

LENGTHS = [0, 1, 2, 15, 16, 17, 255, 256, 257, 1000, 4095, 4096, 3, 4096, 0, 77]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()


def _offsets(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint64)


def _keys(kind, base, ndims, total, rng):
    if kind == "u32":
        space = min(base ** ndims, 2 ** 32)
        return rng.integers(0, space, total, dtype=np.uint64).astype(np.uint32)
    if kind == "u64":
        space = min(base ** ndims, 2 ** 64)
        if space == 2 ** 64:
            return rng.integers(0, 2 ** 64 - 1, total, dtype=np.uint64, endpoint=True)
        return rng.integers(0, space, total, dtype=np.uint64)
    if kind == "fixed_i64":
        return rng.integers(0, base ** ndims, total, dtype=np.int64)
    if kind == "i32":
        return rng.integers(-2 ** 31, 2 ** 31, total, dtype=np.int64).astype(np.int32)
    if kind == "i64":
        return rng.integers(-2 ** 63, 2 ** 63 - 1, total, dtype=np.int64, endpoint=True)
    raise ValueError(kind)


CASES = [
    # kind, base, ndims, descending
    ("u32", 256, 4, False),      # four 8-bit passes: the sub-pass sort
    ("u32", 256, 1, False),      # one pass: the ballot-ranked sort
    ("u32", 10, 6, False),       # 100-cell passes: 7 bits, a 3-bit last sub-pass
    ("u64", 256, 8, False),
    ("u64", 10, 15, False),      # 64-bit division codec
    ("fixed_i64", 10, 9, False),
    ("i32", 256, 4, False),
    ("i64", 16, 16, False),
    ("u32", 256, 4, True),
    ("u32", 10, 6, True),
    ("i64", 256, 8, True),
]


@pytest.mark.parametrize("pairs", [True, False], ids=["pairs", "keys"])
@pytest.mark.parametrize("kind,base,ndims,desc", CASES, ids=[f"{c[0]}-b{c[1]}-n{c[2]}{'-desc' if c[3] else ''}"
                                                               for c in CASES])
def test_small_arrays(kind, base, ndims, desc, pairs):
    import torch
    _say(f"small arrays {kind} base {base} ndims {ndims} desc {desc} pairs {pairs}")
    rng = np.random.default_rng(20210711)
    offs = _offsets(LENGTHS)
    total = int(offs[-1])
    keys = _keys(kind, base, ndims, total, rng)
    # a run of equal keys in one array checks stability on chip
    a = int(offs[11])
    keys[a:a + 3000] = keys[a]
    vals = rng.permutation(total).astype(np.uint32) if pairs else None
    d = B.key_desc(kind, base=base, ndims=ndims, descending=desc)
    kd = api.to_device(keys)
    vd = None if vals is None else api.to_device(vals)
    od = api.to_device(offs)
    ko, vo = api.sort_batched(d, kd, vd, od, len(LENGTHS), total)
    torch.cuda.synchronize()
    gk = api.to_host(ko, key_dtype(kind), key_shape(kind, total))
    gv = None if vd is None else api.to_host(vo, np.uint32, (total,))
    ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind=kind, base=base, ndims=ndims,
                                     groups=fast_groups(kind, base, ndims), descending=desc)
    assert_same(gk, gv, ok, ov, f"{kind} base {base} ndims {ndims} desc {desc}")


LONG_LENGTHS = [4096, 4000, 3001, 2049, 4095, 1, 4096, 2500, 0, 3333]


@pytest.mark.parametrize("kind,base,ndims,desc", CASES, ids=[f"{c[0]}-b{c[1]}-n{c[2]}{'-desc' if c[3] else ''}"
                                                               for c in CASES])
def test_small_arrays_near_the_limit(kind, base, ndims, desc):
    """Arrays averaging over 2048 keys take the ballot-ranked kernel for
    every plan (the sub-pass kernel serves shorter ones)."""
    import torch
    _say(f"small arrays near 4096 {kind} base {base} ndims {ndims} desc {desc}")
    rng = np.random.default_rng(20210712)
    offs = _offsets(LONG_LENGTHS)
    total = int(offs[-1])
    keys = _keys(kind, base, ndims, total, rng)
    keys[int(offs[2]):int(offs[2]) + 2000] = keys[int(offs[2])]
    vals = rng.permutation(total).astype(np.uint32)
    d = B.key_desc(kind, base=base, ndims=ndims, descending=desc)
    ko, vo = api.sort_batched(d, api.to_device(keys), api.to_device(vals), api.to_device(offs), len(LONG_LENGTHS),
                              total)
    torch.cuda.synchronize()
    gk = api.to_host(ko, key_dtype(kind), key_shape(kind, total))
    gv = api.to_host(vo, np.uint32, (total,))
    ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind=kind, base=base, ndims=ndims,
                                     groups=fast_groups(kind, base, ndims), descending=desc)
    assert_same(gk, gv, ok, ov, f"{kind} base {base} ndims {ndims} desc {desc}")


def test_many_small_arrays_log_uniform():
    """Thousands of arrays of 1..4096 keys, every workgroup sorting many."""
    import torch
    _say("many small arrays")
    keys, vals, offs = workloads.batched_u32(count=3000, lo=1, hi=4096)
    total = int(offs[-1])
    d = B.key_desc("u32", base=256, ndims=4)
    ko, vo = api.sort_batched(d, api.to_device(keys), api.to_device(vals), api.to_device(offs.astype(np.uint64)),
                              3000, total)
    torch.cuda.synchronize()
    gk = api.to_host(ko, np.uint32, (total,))
    gv = api.to_host(vo, np.uint32, (total,))
    ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind="u32", base=256, ndims=4, groups=[1, 1, 1, 1])
    assert_same(gk, gv, ok, ov, "3000 log-uniform small arrays")


@pytest.mark.parametrize("n", [1, 2, 17, 1000, 4095, 4096, 4097])
@pytest.mark.parametrize("kind,base,ndims,desc", CASES, ids=[f"{c[0]}-b{c[1]}-n{c[2]}{'-desc' if c[3] else ''}"
                                                               for c in CASES])
def test_single_short_array(kind, base, ndims, desc, n):
    """rs_sort_pairs / rs_sort_keys on one array of at most 4096 keys: one
    workgroup, every pass on chip (4097 takes the passes), also in place."""
    _say(f"short array {kind} base {base} ndims {ndims} desc {desc} n {n}")
    rng = np.random.default_rng(n)
    keys = _keys(kind, base, ndims, n, rng)
    keys[: n // 3] = keys[0]
    vals = rng.permutation(n).astype(np.uint32)
    groups = fast_groups(kind, base, ndims)
    ok, ov, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups, descending=desc)
    gk, gv = gpu_sort(keys, vals, kind, base, ndims, descending=desc)
    assert_same(gk, gv, ok, ov, f"pairs n={n}")
    ok2, _, _ = oracle.sort(keys, None, kind=kind, base=base, ndims=ndims, groups=groups, descending=desc)
    gk2, _ = gpu_sort(keys, None, kind, base, ndims, in_place=True, descending=desc)
    assert_same(gk2, None, ok2, None, f"keys in place n={n}")
