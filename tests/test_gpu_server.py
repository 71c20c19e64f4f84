"""The served request loop on the GPU: every request's result is the same
alone and in the mix (bit for bit), admission refuses what does not fit and
admits it once memory frees up, and a short Poisson trace runs through both
dispatch modes."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads
from paper_2107_01391_amd.serve import Server, make_pool, run_trace
from tests.gpu_helpers import oracle_sort

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()


SIZES = [1, 2, 100, 4095, 4096, 4097, 8191, 8193, 10_000, 65_537, 300_001, 1 << 20]


def _alone(desc, k, v, n):
    """The same request sorted alone by rs_sort_pairs."""
    import torch
    ko, vo = torch.empty_like(k[:n]), torch.empty_like(v[:n])
    tmp = api.empty_device(B.rs_temp_bytes(desc, n, True))
    B.rs_sort_pairs(desc, k, ko, v, vo, n, tmp, tmp.numel())
    torch.cuda.synchronize()
    return ko.cpu().numpy(), vo.cpu().numpy()


@pytest.mark.parametrize("mode,streams,min_batch,batch_max_n", [
    (B.RS_SERVE_BATCHED, 2, 2, 1 << 30), (B.RS_SERVE_BATCHED, 1, 0, 0), (B.RS_SERVE_BATCHED, 2, 0, 5000),
    (B.RS_SERVE_PER_REQUEST, 3, 0, 0)])
def test_mix_equals_alone(mode, streams, min_batch, batch_max_n):
    import torch
    _say(f"server mix vs alone mode={mode} streams={streams}")
    desc = B.key_desc("u32", base=256, ndims=4)
    sizes = np.array(SIZES * 4)
    np.random.default_rng(3).shuffle(sizes)
    pool = make_pool(len(sizes), sizes, seed=99)
    srv = Server(desc, capacity=int(sizes.sum()) + 1000, max_slots=len(sizes), streams=streams, mode=mode,
                 min_batch=min_batch, batch_max_n=batch_max_n)
    try:
        tickets = [srv.submit(k, v) for k, v in pool]
        assert all(t is not None for t in tickets)
        for t in tickets:
            srv.wait(t)
        for i, (t, (k, v)) in enumerate(zip(tickets, pool)):
            rk, rv = srv.result(t)
            n = k.numel()
            gk = rk.view(torch.int32).cpu().numpy()
            gv = rv.cpu().numpy()
            ak, av = _alone(desc, k, v, n)
            assert np.array_equal(gk, ak) and np.array_equal(gv, av), f"request {i} ({n} keys) differs from alone"
            if i < 6:  # and the oracle
                ok, ov = oracle_sort(k.cpu().numpy().view(np.uint32), v.cpu().numpy().view(np.uint32), "u32", 256, 4)
                assert np.array_equal(gk.view(np.uint32), ok) and np.array_equal(gv.view(np.uint32), ov)
            srv.release(t)
        st = srv.stats()
        assert st["completed"] == len(sizes) - 0 and st["keys_sorted"] == int(sizes.sum())
        assert st["p99_ms"] >= st["p50_ms"] > 0
        if mode == B.RS_SERVE_PER_REQUEST:
            assert st["launches"] == len(sizes)
        elif batch_max_n >= 1 << 30:
            assert st["launches"] < len(sizes)  # requests shared launches
    finally:
        srv.close()


def test_admission_by_free_arena_and_slots():
    import torch
    _say("server admission")
    desc = B.key_desc("u32", base=256, ndims=4)
    pool = make_pool(6, np.array([40_000] * 6), seed=5)
    srv = Server(desc, capacity=100_000, max_slots=4, streams=1)
    try:
        t0 = srv.submit(*pool[0])
        t1 = srv.submit(*pool[1])
        assert t0 is not None and t1 is not None
        assert srv.submit(*pool[2]) is None  # 120k keys do not fit 100k
        srv.wait(t0)
        srv.release(t0)
        t2 = srv.submit(*pool[2])  # fits again
        assert t2 is not None
        small = [srv.submit(pool[3][0], pool[3][1], 10) for _ in range(2)]
        assert all(s is not None for s in small)
        assert srv.submit(pool[4][0], pool[4][1], 10) is None  # 4 slots in use
        for t in [t1, t2, *small]:
            srv.wait(t)
        for t, (k, v) in [(t1, pool[1]), (t2, pool[2])]:
            rk, rv = srv.result(t)
            ak, av = _alone(desc, k, v, k.numel())
            assert np.array_equal(rk.view(torch.int32).cpu().numpy(), ak)
            assert np.array_equal(rv.cpu().numpy(), av)
        for t in [t1, t2, *small]:
            srv.release(t)
        assert srv.stats()["busy"] == 2
        with pytest.raises(B.RSError):
            srv.release(t1)  # already released
    finally:
        srv.close()


def test_fixed_point_keys_only_server():
    """8-byte keys, three passes, no values: the mix still equals alone."""
    import torch
    _say("server fixed point keys only")
    desc = B.key_desc("fixed_i64", base=10, ndims=9, frac_digits=3)
    w = workloads.fixed_point_decimals(500_000)
    cuts = [0, 1, 5000, 5001, 70_000, 200_000, 500_000]
    reqs = [api.to_device(w.keys[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
    srv = Server(desc, capacity=600_000, max_slots=16, streams=2, with_values=False)
    try:
        tickets = [srv.submit(k, None, k.numel() // 8) for k in reqs]
        for t in tickets:
            srv.wait(t)
        for t, k, (a, b) in zip(tickets, reqs, zip(cuts[:-1], cuts[1:])):
            rk, _ = srv.result(t)
            got = rk.cpu().numpy().view(np.int64)
            ok, _ = oracle_sort(w.keys[a:b], None, "fixed_i64", 10, 9)
            assert np.array_equal(got, ok)
            srv.release(t)
    finally:
        srv.close()


@pytest.mark.parametrize("mode", [B.RS_SERVE_BATCHED, B.RS_SERVE_PER_REQUEST])
def test_signed_descending_server(mode):
    """Signed 32-bit keys in descending order with values, submitted
    together: each result equals the oracle's sort of that request."""
    _say(f"server signed descending mode={mode}")
    desc = B.key_desc("i32", base=256, ndims=4, descending=True)
    rng = np.random.default_rng(77)
    sizes = [1, 4096, 4097, 30_000, 250_000, 3, 70_001]
    keys = [rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32) for n in sizes]
    for k in keys[3:4]:
        k[::5] = k[0]  # ties
    vals = [rng.permutation(n).astype(np.uint32) for n in sizes]
    srv = Server(desc, capacity=400_000, max_slots=16, streams=2, mode=mode)
    try:
        dev = [(api.to_device(k), api.to_device(v)) for k, v in zip(keys, vals)]  # alive until the end
        tickets = [srv.submit(dk, dv, k.shape[0]) for (dk, dv), k in zip(dev, keys)]
        assert srv.held() == len(tickets)
        for t in tickets:
            srv.wait(t)
        for t, k, v in zip(tickets, keys, vals):
            rk, rv = srv.result(t)
            ok, ov = oracle_sort(k, v, "i32", 256, 4, descending=True)
            assert np.array_equal(rk.cpu().numpy().view(np.int32), ok)
            assert np.array_equal(rv.cpu().numpy().view(np.uint32), ov)
            srv.release(t)
        assert srv.held() == 0
    finally:
        srv.close()


@pytest.mark.parametrize("mode", [B.RS_SERVE_BATCHED, B.RS_SERVE_PER_REQUEST])
def test_submit_temporaries(mode):
    """Requests submitted as temporaries that the caller drops at once,
    while new tensors are allocated and written on torch's stream: the
    server holds each request's sources until it is released, so every
    result is still the sort of its own request."""
    _say(f"server temporaries mode={mode}")
    import torch
    desc = B.key_desc("u32", base=256, ndims=4)
    rng = np.random.default_rng(78)
    sizes = [4097, 1, 30_000, 4096, 250_000, 70_001, 5, 100_000]
    keys = [rng.integers(0, 2**32, n, dtype=np.uint32) for n in sizes]
    vals = [rng.permutation(n).astype(np.uint32) for n in sizes]
    srv = Server(desc, capacity=600_000, max_slots=16, streams=2, mode=mode)
    try:
        tickets = []
        for k, v in zip(keys, vals):
            tickets.append(srv.submit(api.to_device(k), api.to_device(v), k.shape[0]))
            # blocks a freed source would be handed to: overwrite them now
            junk = torch.full((300_000,), -1, dtype=torch.int32, device="cuda")
            del junk
        assert srv.held() == len(tickets)
        for t in tickets:
            srv.wait(t)
        for t, k, v in zip(tickets, keys, vals):
            rk, rv = srv.result(t)
            ok, ov = oracle_sort(k, v, "u32", 256, 4)
            assert np.array_equal(rk.cpu().numpy().view(np.uint32), ok)
            assert np.array_equal(rv.cpu().numpy().view(np.uint32), ov)
            srv.release(t)
        assert srv.held() == 0
    finally:
        srv.close()


@pytest.mark.parametrize("mode", [B.RS_SERVE_BATCHED, B.RS_SERVE_PER_REQUEST])
def test_short_poisson_trace(mode):
    _say(f"server trace mode={mode}")
    desc = B.key_desc("u32", base=256, ndims=4)
    sizes = workloads.batched_sizes(120, lo=1024, hi=1 << 18)
    pool = make_pool(16, sizes[:16], seed=11)
    gaps = np.random.default_rng(1).exponential(1 / 2000.0, 120)
    srv = Server(desc, capacity=1 << 24, max_slots=128, streams=2, mode=mode)
    try:
        st = run_trace(srv, pool, gaps, sizes, warmup=20)
    finally:
        srv.close()
    assert st["completed"] == 100
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
