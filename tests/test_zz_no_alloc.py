"""rs_sort_pairs_noalloc (the pair sort on the library's static device
scratch) against rs_sort_pairs on a caller's scratch, bit for bit, on calls
in a row that share the one static array: each later call smaller than the
one before, so that it runs on what the earlier call left there."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    B.rs_tuning_clear()


def _both(d, keys, vals, kind_dtype, shape):
    """(noalloc keys, values), (rs_sort_pairs keys, values) as host arrays."""
    import torch
    n = vals.shape[0]
    kd, vd = api.to_device(keys), api.to_device(vals)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    B.rs_sort_pairs_noalloc(d, kd, ko, vd, vo, n)
    torch.cuda.synchronize()
    got = (api.to_host(ko, kind_dtype, shape), api.to_host(vo, np.uint32, (n,)))
    rk, rv = api.sort_pairs(d, kd, vd, n)
    torch.cuda.synchronize()
    ref = (api.to_host(rk, kind_dtype, shape), api.to_host(rv, np.uint32, (n,)))
    return got, ref


# sizes in decreasing order: prescanned passes, chained passes, one workgroup
@pytest.mark.parametrize("sizes", [(8_000_000, 1_000_003, 77_777, 4096, 1)])
def test_noalloc_equals_caller_scratch_u32(sizes):
    d = B.key_desc("u32", base=256, ndims=4)
    for n in sizes:
        _say(f"noalloc u32 pairs n={n}")
        w = workloads.uniform_u32_pairs(n, seed_extra=(n,))
        got, ref = _both(d, w.keys, w.vals, np.uint32, (n,))
        assert np.array_equal(got[0], ref[0]), f"n={n}: keys differ"
        assert np.array_equal(got[1], ref[1]), f"n={n}: values differ"
        # and the sort itself: non-decreasing, ties in input order
        k, v = got
        assert np.all(k[1:] >= k[:-1]) and np.array_equal(w.keys[v], k)
        same = k[1:] == k[:-1]
        assert np.all(v[1:][same] > v[:-1][same])


def test_noalloc_strings_then_smaller_fixed_point():
    d = B.key_desc("str", base=27, ndims=16)
    w = workloads.strings16(2_300_000, seed_extra=(5,))
    _say("noalloc strings n=2300000")
    got, ref = _both(d, w.keys, w.vals, np.uint8, (w.n, 16))
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    d = B.key_desc("fixed_i64", base=10, ndims=9, frac_digits=3)
    w = workloads.fixed_point_decimals(500_000, seed_extra=(6,))
    _say("noalloc fixed point n=500000")
    got, ref = _both(d, w.keys, w.vals, np.int64, (w.n,))
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_noalloc_refuses_beyond_the_static_scratch():
    import torch
    d = B.key_desc("u32", base=256, ndims=4)
    n = 9_000_000
    kd = torch.zeros(n * 4, dtype=torch.uint8, device="cuda")
    vd = torch.zeros(n * 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.RSError) as e:
        B.rs_sort_pairs_noalloc(d, kd, kd, vd, vd, n)
    assert e.value.status == 5
    torch.cuda.synchronize()
    assert int(kd.sum()) == 0  # nothing ran
