"""Batched form: many independent arrays in one launch sequence, each equal
to the oracle's sort of that array alone; and the sequence captured in a
hipGraph, replayed several times, equal to the eager result every time."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads
from tests.gpu_helpers import fast_groups, key_dtype, key_shape

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()


def gpu_batched(keys, vals, offs, kind, base, ndims, in_place=False):
    import torch
    nseg = offs.shape[0] - 1
    total = int(offs[-1])
    d = B.key_desc(kind, base=base, ndims=ndims)
    kd = api.to_device(keys)
    vd = None if vals is None else api.to_device(vals)
    od = api.to_device(offs.astype(np.uint64))
    ko = kd if in_place else None
    vo = vd if in_place else None
    ko, vo = api.sort_batched(d, kd, vd, od, nseg, total, keys_out=ko, vals_out=vo)
    torch.cuda.synchronize()
    gk = api.to_host(ko, key_dtype(kind), key_shape(kind, total))
    gv = None if vd is None else api.to_host(vo, np.uint32, (total,))
    return gk, gv


def oracle_batched(keys, vals, offs, kind, base, ndims):
    ok, ov, _ = oracle.sort_segments(keys, vals, offs, kind=kind, base=base, ndims=ndims,
                                     groups=fast_groups(kind, base, ndims))
    return ok, ov


def _cmp(gk, gv, ok, ov, offs):
    for i in range(offs.shape[0] - 1):
        a, b = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(gk[a:b], ok[a:b]), f"array {i} ({b - a} keys): keys differ"
        if ov is not None:
            assert np.array_equal(gv[a:b], ov[a:b]), f"array {i} ({b - a} keys): values differ"


@pytest.fixture(params=[256, 512], ids=["tile256", "tile512"])
def tile_block(request, monkeypatch):
    """Both tile widths of the large arrays' passes (4096 and 8192 keys)."""
    monkeypatch.setenv("RS_TILE_BLOCK", str(request.param))
    yield request.param


@pytest.mark.parametrize("count,lo,hi", [(1, 1, 1), (1, 5000, 5000), (7, 1, 300), (64, 1, 40_000),
                                         (300, 1024, 65_536), (16, 100_000, 400_000)])
def test_batched_u32_pairs(tile_block, count, lo, hi):
    _say(f"batched u32 pairs count={count} sizes [{lo}, {hi}]")
    keys, vals, offs = workloads.batched_u32(count=count, lo=lo, hi=hi)
    gk, gv = gpu_batched(keys, vals, offs, "u32", 256, 4)
    ok, ov = oracle_batched(keys, vals, offs, "u32", 256, 4)
    _cmp(gk, gv, ok, ov, offs)


def test_batched_with_empty_and_single_arrays(tile_block):
    _say(f"batched with empty arrays, tile block {tile_block}")
    sizes = np.array([0, 1, 0, 4096, 4097, 0, 2, 12_000, 0, 8192, 8193, 16_384, 24_577], np.int64)
    offs = np.zeros(sizes.shape[0] + 1, np.uint64)
    offs[1:] = np.cumsum(sizes)
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 2**32, int(offs[-1]), dtype=np.uint32)
    vals = np.concatenate([np.arange(s, dtype=np.uint32) for s in sizes])
    gk, gv = gpu_batched(keys, vals, offs, "u32", 256, 4)
    ok, ov = oracle_batched(keys, vals, offs, "u32", 256, 4)
    _cmp(gk, gv, ok, ov, offs)


def test_batched_keys_only(tile_block):
    _say("batched keys only")
    keys, _, offs = workloads.batched_u32(count=40, lo=10, hi=30_000)
    gk, _ = gpu_batched(keys, None, offs, "u32", 256, 4)
    ok, _ = oracle_batched(keys, None, offs, "u32", 256, 4)
    _cmp(gk, None, ok, None, offs)


def test_batched_in_place():
    _say("batched in place")
    keys, vals, offs = workloads.batched_u32(count=20, lo=100, hi=50_000)
    gk, gv = gpu_batched(keys, vals, offs, "u32", 256, 4, in_place=True)
    ok, ov = oracle_batched(keys, vals, offs, "u32", 256, 4)
    _cmp(gk, gv, ok, ov, offs)


def test_batched_fixed_point_and_strings(tile_block):
    _say("batched fixed point")
    w = workloads.fixed_point_decimals(60_000)
    offs = np.array([0, 10, 4000, 4100, 30_000, 60_000], np.uint64)
    gk, gv = gpu_batched(w.keys, w.vals, offs, "fixed_i64", 10, 9)
    ok, ov = oracle_batched(w.keys, w.vals, offs, "fixed_i64", 10, 9)
    _cmp(gk, gv, ok, ov, offs)
    _say("batched strings")
    w = workloads.strings16(20_000)
    offs = np.array([0, 1, 2048, 2049, 9000, 20_000], np.uint64)
    gk, gv = gpu_batched(w.keys, w.vals, offs, "str", 27, 16)
    ok, ov = oracle_batched(w.keys, w.vals, offs, "str", 27, 16)
    _cmp(gk, gv, ok, ov, offs)


def test_batched_equals_per_array_calls():
    """The batched launch gives the same bytes as rs_sort_pairs per array."""
    import torch
    _say("batched == per array")
    keys, vals, offs = workloads.batched_u32(count=24, lo=1000, hi=100_000)
    gk, gv = gpu_batched(keys, vals, offs, "u32", 256, 4)
    d = B.key_desc("u32", base=256, ndims=4)
    for i in range(offs.shape[0] - 1):
        a, b = int(offs[i]), int(offs[i + 1])
        ko, vo = api.sort_pairs(d, api.to_device(keys[a:b]), api.to_device(vals[a:b]), b - a)
        torch.cuda.synchronize()
        assert np.array_equal(api.to_host(ko, np.uint32, (b - a,)), gk[a:b])
        assert np.array_equal(api.to_host(vo, np.uint32, (b - a,)), gv[a:b])


def test_batched_graph_replay():
    """Capture the batched sequence once; replay it three times with other
    work and synchronisations between replays; every replay equals eager."""
    import torch
    _say("batched graph replay")
    keys, vals, offs = workloads.batched_u32(count=50, lo=500, hi=60_000)
    nseg, total = offs.shape[0] - 1, int(offs[-1])
    d = B.key_desc("u32", base=256, ndims=4)
    kd, vd, od = api.to_device(keys), api.to_device(vals), api.to_device(offs)
    ko, vo = api.empty_device(kd.numel()), api.empty_device(vd.numel())
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, total, nseg, True))
    B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    eager_k, eager_v = ko.clone(), vo.clone()
    ok, ov = oracle_batched(keys, vals, offs, "u32", 256, 4)
    _cmp(api.to_host(eager_k, np.uint32, (total,)), api.to_host(eager_v, np.uint32, (total,)), ok, ov, offs)

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel(), s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        ko.zero_()
        vo.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # other eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(ko, eager_k) and torch.equal(vo, eager_v), f"replay {rep} differs from eager"


@pytest.mark.parametrize("offs", [[0, 5, 3, 10], [1, 5, 7, 10], [0, 5, 7, 9]])
def test_batched_validate_rejects_bad_offsets(offs):
    """Decreasing offsets, a first offset other than 0, a last one other than
    total: refused before any sort kernel runs (only with validation; the
    offsets are never sorted with)."""
    import torch
    _say(f"batched validate offsets {offs}")
    d = B.key_desc("u32", base=256, ndims=4, validate=True)
    keys = np.arange(10, dtype=np.uint32)[::-1].copy()
    kd, vd = api.to_device(keys), api.to_device(np.arange(10, dtype=np.uint32))
    od = api.to_device(np.array(offs, np.uint64))
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, 10, 3, True))
    with pytest.raises(B.RSError) as e:
        B.rs_sort_batched(d, kd, ko, vd, vo, od, 3, 10, tmp, tmp.numel())
    assert e.value.status == 2 and "offsets" in str(e.value)
    od.copy_(torch.from_numpy(np.array([0, 3, 3, 10], np.uint64).view(np.uint8)).cuda())
    B.rs_sort_batched(d, kd, ko, vd, vo, od, 3, 10, tmp, tmp.numel())
    torch.cuda.synchronize()
    got = api.to_host(ko, np.uint32, (10,))
    assert got.tolist() == sorted(keys[:3].tolist()) + sorted(keys[3:].tolist())


@pytest.mark.parametrize("offs", [[0, 20_000, 5_000, 60_000, 1 << 40, 3, 50_000],
                                  [0, 50_000, 0, 50_000, 0, 50_000, 0],
                                  [7, 3, (1 << 64) - 1, 0, 49_999, 50_000, 50_000]])
def test_batched_bad_offsets_stay_in_bounds(offs, tile_block):
    """Without validation, offsets that decrease, overlap or point past the
    end give an unspecified order but no access outside the buffers: the
    arrays' bounds are clamped on the device before any kernel reads keys
    (overlapping arrays also have their tiles cut at the scratch's bound).
    The outputs sit between guard bands that must come back untouched, and
    the same scratch then sorts valid offsets correctly."""
    import torch
    _say(f"batched bad offsets {offs} tile_block={tile_block}")
    total, nseg, guard = 50_000, len(offs) - 1, 1 << 16
    d = B.key_desc("u32", base=256, ndims=4)
    keys, vals, good = workloads.batched_u32(count=nseg, lo=1000, hi=20_000)
    keys = np.resize(keys, total).astype(np.uint32)
    vals = np.arange(total, dtype=np.uint32)
    kd, vd = api.to_device(keys), api.to_device(vals)
    kbuf = torch.full((total + 2 * guard,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    vbuf = torch.full((total + 2 * guard,), 0x3C3C3C3C, dtype=torch.int32, device="cuda")
    ko, vo = kbuf[guard:guard + total], vbuf[guard:guard + total]
    tmp = api.empty_device(B.rs_batched_temp_bytes(d, total, nseg, True))
    od = api.to_device(np.array(offs, dtype=np.uint64))
    B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    for buf, fill in ((kbuf, 0x5A5A5A5A), (vbuf, 0x3C3C3C3C)):
        assert bool((buf[:guard] == fill).all()) and bool((buf[guard + total:] == fill).all()), "guard band written"
    # the same scratch, valid offsets
    goff = np.linspace(0, total, nseg + 1).astype(np.uint64)
    od = api.to_device(goff)
    B.rs_sort_batched(d, kd, ko, vd, vo, od, nseg, total, tmp, tmp.numel())
    torch.cuda.synchronize()
    gk, gv = ko.cpu().numpy().view(np.uint32), vo.cpu().numpy().view(np.uint32)
    ok, ov = oracle_batched(keys, vals, goff, "u32", 256, 4)
    _cmp(gk, gv, ok, ov, goff)
