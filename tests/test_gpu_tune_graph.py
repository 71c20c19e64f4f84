"""The autotuner and captured-graph replays on the GPU: whatever choice the
tuner keeps, and however often a captured sort is replayed with new data,
the output stays the oracle's."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads
from tests.gpu_helpers import assert_same, oracle_sort

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
    yield
    B.rs_tuning_clear()


@pytest.mark.parametrize("base,ndims,n", [(256, 4, 1 << 20), (2, 32, 300_001), (16, 8, 5 << 20)])
def test_tune_sort_keeps_a_choice_and_results_stay_exact(base, ndims, n):
    import torch
    _say(f"tune u32 base {base} n={n}")
    w = workloads.uniform_u32_pairs(n)
    d = B.key_desc("u32", base=base, ndims=ndims)
    ki, vi = api.to_device(w.keys), api.to_device(w.vals)
    ko, vo = api.empty_device(ki.numel()), api.empty_device(vi.numel())
    need = B.rs_tune_temp_bytes(d, n, 0, True)
    tmp = api.empty_device(need)
    best, ms = B.rs_tune_sort(d, ki, ko, vi, vo, n, tmp, need, reps=2)
    assert ms > 0
    assert B.rs_tuning_get(d, n, True).as_dict() == best.as_dict()
    # the tuner's own outputs and a plain sort with the kept choice
    ok, ov = oracle_sort(w.keys, w.vals, "u32", base, ndims)
    torch.cuda.synchronize()
    assert_same(api.to_host(ko, np.uint32, (n,)), api.to_host(vo, np.uint32, (n,)), ok, ov, "tuner output")
    ko.zero_()
    vo.zero_()
    B.rs_sort_pairs(d, ki, ko, vi, vo, n, tmp, need)
    torch.cuda.synchronize()
    assert_same(api.to_host(ko, np.uint32, (n,)), api.to_host(vo, np.uint32, (n,)), ok, ov, f"kept {best.as_dict()}")
    # inputs untouched
    assert np.array_equal(api.to_host(ki, np.uint32, (n,)), w.keys)


def test_tune_fixed_point_and_batched():
    import torch
    _say("tune fixed point")
    w = workloads.fixed_point_decimals(400_003)
    n = w.keys.shape[0]
    d = B.key_desc("fixed_i64", base=10, ndims=9, frac_digits=3)
    ki, vi = api.to_device(w.keys), api.to_device(w.vals)
    ko, vo = api.empty_device(ki.numel()), api.empty_device(vi.numel())
    tmp = api.empty_device(B.rs_tune_temp_bytes(d, n, 0, True))
    best, _ = B.rs_tune_sort(d, ki, ko, vi, vo, n, tmp, tmp.numel(), reps=1)
    assert best.max_cells in (10, 100, 1000)
    torch.cuda.synchronize()
    ok, ov = oracle_sort(w.keys, w.vals, "fixed_i64", 10, 9)
    assert_same(api.to_host(ko, np.int64, (n,)), api.to_host(vo, np.uint32, (n,)), ok, ov)

    _say("tune batched")
    keys, vals, offs = workloads.batched_u32(count=40, lo=100, hi=200_000)
    total = int(offs[-1])
    d = B.key_desc("u32", base=256, ndims=4)
    ki, vi, od = api.to_device(keys), api.to_device(vals), api.to_device(offs)
    ko, vo = api.empty_device(ki.numel()), api.empty_device(vi.numel())
    tmp = api.empty_device(B.rs_tune_temp_bytes(d, total, 40, True))
    best, _ = B.rs_tune_batched(d, ki, ko, vi, vo, od, 40, total, tmp, tmp.numel(), reps=1)
    assert B.rs_tuning_get(d, total, True, batched=True).as_dict() == best.as_dict()
    ko.zero_()
    B.rs_sort_batched(d, ki, ko, vi, vo, od, 40, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    ok, ov, _ = __import__("oracle").sort_segments(keys, vals, offs, kind="u32", base=256, ndims=4,
                                                   groups=[1, 1, 1, 1])
    assert np.array_equal(api.to_host(ko, np.uint32, (total,)), ok)
    assert np.array_equal(api.to_host(vo, np.uint32, (total,)), ov)


@pytest.mark.parametrize("n,prescan", [(100_003, False), (3 << 20, True)])
def test_graph_sort_replays_new_data(monkeypatch, n, prescan):
    """Capture once; before every replay rewrite the keys (eager work and a
    synchronisation in between); every replay must match the oracle."""
    import torch
    monkeypatch.setenv("RS_PRESCAN_MIN_N", "1" if prescan else str(1 << 40))
    _say(f"graph sort n={n} prescan={prescan}")
    d = B.key_desc("u32", base=256, ndims=4)
    ki = api.empty_device(4 * n)
    vi = api.empty_device(4 * n)
    ko, vo = api.empty_device(4 * n), api.empty_device(4 * n)
    tmp = api.empty_device(B.rs_temp_bytes(d, n, True))
    g = B.rs_graph_sort(d, ki, ko, vi, vo, n, tmp, tmp.numel())
    try:
        for rep in range(3):
            w = workloads.uniform_u32_pairs(n, seed_extra=[rep])
            ki.copy_(torch.from_numpy(w.keys.view(np.uint8)).cuda())
            vi.copy_(torch.from_numpy(w.vals.view(np.uint8)).cuda())
            ko.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            ok, ov = oracle_sort(w.keys, w.vals, "u32", 256, 4)
            assert_same(api.to_host(ko, np.uint32, (n,)), api.to_host(vo, np.uint32, (n,)), ok, ov, f"replay {rep}")
    finally:
        g.close()


@pytest.mark.parametrize("prescan", [False, True], ids=["chained", "prescanned_narrowed"])
def test_graph_keys_only_in_place_odd_passes(monkeypatch, prescan):
    """Keys only, in place, an odd pass count: chained, the graph holds the
    copy kernel that starts an odd pass count in place; prescanned, the
    fixed-point keys (below 10^9) are narrowed to 32-bit words, sorted and
    widened back in place."""
    import torch
    monkeypatch.setenv("RS_PRESCAN_MIN_N", "1" if prescan else str(1 << 40))
    _say(f"graph keys only in place prescan={prescan}")
    n = 200_001
    d = B.key_desc("fixed_i64", base=10, ndims=9, frac_digits=3)
    k = api.empty_device(8 * n)
    tmp = api.empty_device(B.rs_temp_bytes(d, n, False))
    g = B.rs_graph_sort(d, k, k, None, None, n, tmp, tmp.numel())
    try:
        for rep in range(3):
            w = workloads.fixed_point_decimals(n, seed_extra=[rep])
            k.copy_(torch.from_numpy(w.keys.view(np.uint8)).cuda())
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            ok, _ = oracle_sort(w.keys, None, "fixed_i64", 10, 9)
            assert np.array_equal(api.to_host(k, np.int64, (n,)), ok), f"replay {rep}"
    finally:
        g.close()


def test_graph_batched_replays_new_boundaries():
    """The batched graph depends only on (total, nseg): new keys and new
    array boundaries before every replay."""
    import oracle
    import torch
    _say("graph batched")
    nseg, total = 64, 1_500_000
    d = B.key_desc("u32", base=256, ndims=4)
    ki, vi = api.empty_device(4 * total), api.empty_device(4 * total)
    ko, vo = api.empty_device(4 * total), api.empty_device(4 * total)
    od = api.empty_device(8 * (nseg + 1))
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, total, nseg, True))
    g = B.rs_graph_sort_batched(d, ki, ko, vi, vo, od, nseg, total, tmp, tmp.numel())
    try:
        rng = np.random.default_rng(77)
        for rep in range(3):
            cuts = np.sort(rng.integers(0, total + 1, nseg - 1))
            if rep == 1:
                cuts[:10] = 0  # empty arrays
            offs = np.concatenate([[0], cuts, [total]]).astype(np.uint64)
            keys = rng.integers(0, 2**32, total, dtype=np.uint32)
            vals = np.arange(total, dtype=np.uint32)
            ki.copy_(torch.from_numpy(keys.view(np.uint8)).cuda())
            vi.copy_(torch.from_numpy(vals.view(np.uint8)).cuda())
            od.copy_(torch.from_numpy(offs.view(np.uint8)).cuda())
            ko.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind="u32", base=256, ndims=4, groups=[1, 1, 1, 1])
            assert np.array_equal(api.to_host(ko, np.uint32, (total,)), ok), f"replay {rep} keys"
            assert np.array_equal(api.to_host(vo, np.uint32, (total,)), ov), f"replay {rep} values"
    finally:
        g.close()
