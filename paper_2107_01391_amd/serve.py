"""Served request loop (rs_server, C++) from Python, and a trace driver.

A Server owns nothing but the C handle: its device arenas and scratch are
torch tensors allocated here and kept alive with it.  run_trace() replays an
arrival trace (seeded Poisson arrivals, log-uniform sizes) against a server,
submitting each request at its arrival time, retrying while admission says
busy, and releasing each result once done; it returns the server's latency
statistics and throughput.

    python -m paper_2107_01391_amd.serve --rates 500,1000,2000,4000,8000,0 --requests 2000
"""
from __future__ import annotations

import argparse
import ctypes
import json
import time

import numpy as np

from . import _binding as B


class Server:
    def __init__(self, desc: B.KeyDesc, capacity: int, max_slots: int = 256, streams: int = 2,
                 mode: int = B.RS_SERVE_BATCHED, with_values: bool = True, max_batch: int = 0):
        import torch
        B.load_library()
        self.desc = desc
        self.cfg = B.ServerConfig(capacity, max_slots, max_batch, streams, mode, int(bool(with_values)), 0)
        kb = {0: 4, 1: 8, 2: 8, 3: 16}[desc.kind]
        self.kb = kb
        dev = "cuda"
        self.keys_in = torch.empty(capacity * kb, dtype=torch.uint8, device=dev)
        self.keys_out = torch.empty(capacity * kb, dtype=torch.uint8, device=dev)
        self.vals_in = torch.empty(capacity if with_values else 0, dtype=torch.int32, device=dev)
        self.vals_out = torch.empty(capacity if with_values else 0, dtype=torch.int32, device=dev)
        need = ctypes.c_size_t(0)
        lib = B.load_library()
        B._check(lib.rs_server_work_bytes(ctypes.byref(desc), ctypes.byref(self.cfg), ctypes.byref(need)))
        self.work = torch.empty(need.value, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        h = ctypes.c_void_p(None)
        vi = self.vals_in.data_ptr() if with_values else None
        vo = self.vals_out.data_ptr() if with_values else None
        B._check(lib.rs_server_create(ctypes.byref(desc), ctypes.byref(self.cfg), self.keys_in.data_ptr(),
                                      self.keys_out.data_ptr(), vi, vo, self.work.data_ptr(), need.value,
                                      ctypes.byref(h)))
        self._h = h.value

    @staticmethod
    def clock() -> int:
        t = ctypes.c_uint64(0)
        B._check(B.load_library().rs_server_clock(ctypes.byref(t)))
        return t.value

    def submit(self, keys, vals=None, n: int | None = None, arrival_ns: int = 0) -> int | None:
        """Ticket, or None when admission refuses the request now (busy)."""
        lib = B.load_library()
        n = keys.numel() if n is None else n
        t = ctypes.c_uint64(0)
        st = lib.rs_server_submit(self._h, B._ptr(keys), B._ptr(vals), n, arrival_ns, ctypes.byref(t))
        if st == B.RS_ERR_BUSY:
            return None
        B._check(st)
        return t.value

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        B._check(B.load_library().rs_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> None:
        B._check(B.load_library().rs_server_wait(self._h, ticket))

    def result(self, ticket: int):
        """(keys bytes, values) views of the output arena for a done request."""
        off, n = ctypes.c_uint64(0), ctypes.c_uint64(0)
        B._check(B.load_library().rs_server_result(self._h, ticket, ctypes.byref(off), ctypes.byref(n)))
        o, m = off.value, n.value
        k = self.keys_out[o * self.kb:(o + m) * self.kb]
        v = self.vals_out[o:o + m] if self.cfg.with_values else None
        return k, v

    def release(self, ticket: int) -> None:
        B._check(B.load_library().rs_server_release(self._h, ticket))

    def stats(self) -> dict:
        s = B.ServerStats()
        B._check(B.load_library().rs_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self) -> None:
        B._check(B.load_library().rs_server_reset_stats(self._h))

    def close(self) -> None:
        if self._h:
            B._check(B.load_library().rs_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_pool(count: int, sizes: np.ndarray, seed: int):
    """`count` distinct device request arrays (u32 keys, local-index values)
    whose sizes cycle through `sizes`; drawn on the device, seeded."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    pool = []
    for i in range(count):
        n = int(sizes[i % len(sizes)])
        k = torch.randint(0, 2**32, (n,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
        v = torch.arange(n, dtype=torch.int32, device="cuda")
        pool.append((k, v))
    torch.cuda.synchronize()
    return pool


def run_trace(server: Server, pool, gaps_s: np.ndarray, sizes: np.ndarray, warmup: int = 0) -> dict:
    """Submits request i (pool entry i mod len(pool), its first sizes[i]
    keys) at arrival time sum(gaps[:i+1]); all-zero gaps submit as fast as
    admission allows.  A refused (busy) request is retried after the oldest
    outstanding one completes; its latency still counts from its arrival.
    Done requests are released as soon as they are seen.  Statistics cover
    the requests after the first `warmup`."""
    count = len(gaps_s)
    t0 = Server.clock()
    arrivals = t0 + np.cumsum(gaps_s * 1e9).astype(np.int64)
    pending: list[int] = []
    i = 0
    while i < count or pending:
        if pending:
            still = []
            for t in pending:
                if server.done(t):
                    server.release(t)
                else:
                    still.append(t)
            pending = still
        if i < count and Server.clock() >= arrivals[i]:
            k, v = pool[i % len(pool)]
            n = int(min(sizes[i], k.numel()))
            t = server.submit(k, v, n, int(arrivals[i]))
            if t is None:
                if not pending:
                    raise RuntimeError("request refused with nothing outstanding: arena or slots too small")
                server.wait(pending[0])
                continue
            pending.append(t)
            i += 1
            if i == warmup:
                for t in pending:
                    server.wait(t)
                    server.release(t)
                pending = []
                server.reset_stats()
            continue
        wait_s = 20e-6 if i >= count else min(20e-6, max(0.0, (arrivals[i] - Server.clock()) / 1e9))
        if wait_s > 0:
            time.sleep(wait_s)
    st = server.stats()
    st["gkeys_per_s"] = st["keys_sorted"] / (st["span_ms"] / 1e3) / 1e9 if st["span_ms"] > 0 else 0.0
    return st


def sweep(rates, requests: int, warmup: int, capacity: int, streams: int, seed: int = 20210708) -> list[dict]:
    from . import workloads
    desc = B.key_desc("u32", base=256, ndims=4)
    rows = []
    sizes_all = workloads.batched_sizes(requests + warmup, seed_extra=[seed])
    pool = make_pool(64, sizes_all[:64], seed)
    for mode, name in ((B.RS_SERVE_PER_REQUEST, "per_request"), (B.RS_SERVE_BATCHED, "batched")):
        srv = Server(desc, capacity, max_slots=512, streams=streams, mode=mode)
        try:
            for rate in rates:
                rng = np.random.default_rng([seed, int(rate)])
                gaps = rng.exponential(1.0 / rate, requests + warmup) if rate > 0 else np.zeros(requests + warmup)
                st = run_trace(srv, pool, gaps, sizes_all, warmup=warmup)
                st.update({"mode": name, "rate": rate})
                rows.append(st)
                print(json.dumps(st), flush=True)
        finally:
            srv.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="500,1000,2000,4000,8000,0")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--capacity", type=int, default=1 << 30)
    ap.add_argument("--streams", type=int, default=2)
    a = ap.parse_args()
    sweep([float(r) for r in a.rates.split(",")], a.requests, a.warmup, a.capacity, a.streams)


if __name__ == "__main__":
    main()
