"""Served request loop (rs_server, C++) from Python, and a trace driver.

A Server owns the C handle; its device arenas and scratch are torch tensors
allocated here and kept alive with it.  The server copies a request's keys
and values into its arena on its own upload stream, after submit() has
returned, so submit() keeps a reference to the tensors it was given until
the request is released (or the server closed): a caller may pass
temporaries, and torch's allocator cannot hand their memory to another
tensor while the copy may still read it.  The copy also waits for the work
already enqueued on torch's current stream, where the sources were written.
run_trace() replays an
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
                 mode: int = B.RS_SERVE_BATCHED, with_values: bool = True, max_batch: int = 0,
                 min_batch: int = 0, batch_max_n: int = 0):
        import torch
        B.load_library()
        self.desc = desc
        self.cfg = B.ServerConfig(capacity, max_slots, max_batch, streams, mode, int(bool(with_values)), min_batch,
                                  batch_max_n)
        kb = {B.RS_KEY_U32: 4, B.RS_KEY_U64: 8, B.RS_KEY_FIXED_I64: 8, B.RS_KEY_STR: desc.str_width or 16,
              B.RS_KEY_I32: 4, B.RS_KEY_I64: 8}[desc.kind]
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
        self._held = {}  # ticket -> the submitted source tensors, until release

    @staticmethod
    def clock() -> int:
        t = ctypes.c_uint64(0)
        B._check(B.load_library().rs_server_clock(ctypes.byref(t)))
        return t.value

    def submit(self, keys, vals=None, n: int | None = None, arrival_ns: int = 0) -> int | None:
        """Ticket, or None when admission refuses the request now (busy).
        keys / vals (tensors) are held until the ticket is released."""
        import torch
        lib = B.load_library()
        n = keys.numel() if n is None else n
        t = ctypes.c_uint64(0)
        src_stream = torch.cuda.current_stream().cuda_stream if getattr(keys, "is_cuda", False) else None
        st = lib.rs_server_submit(self._h, B._ptr(keys), B._ptr(vals), n, arrival_ns, src_stream, ctypes.byref(t))
        if st == B.RS_ERR_BUSY:
            return None
        B._check(st)
        self._held[t.value] = (keys, vals)
        return t.value

    def held(self) -> int:
        """Requests whose source tensors are still referenced."""
        return len(self._held)

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        B._check(B.load_library().rs_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> None:
        B._check(B.load_library().rs_server_wait(self._h, ticket))

    def collect(self, wait_us: int = 0, max_n: int = 1024) -> list[int]:
        """Tickets finished since the last collect (waits up to wait_us for one)."""
        buf = (ctypes.c_uint64 * max_n)()
        k = ctypes.c_uint32(0)
        B._check(B.load_library().rs_server_collect(self._h, buf, max_n, ctypes.byref(k), wait_us))
        return list(buf[:k.value])

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
        self._held.pop(ticket, None)

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
        self._held.clear()  # destroy has waited for every upload

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_pool(count: int, sizes: np.ndarray, seed: int):
    """`count` distinct device request arrays (u32 keys, local-index values)
    whose sizes cycle through `sizes`; drawn on the device, seeded.  A trace
    request takes the first sizes[i] keys of its pool entry."""
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
    admission allows.  A refused (busy) request is retried once another one
    completes; its latency still counts from its arrival.  Finished requests
    are collected and released as they complete.  Statistics cover the
    requests after the first `warmup`."""
    count = len(gaps_s)
    t0 = Server.clock()
    arrivals = t0 + np.cumsum(gaps_s * 1e9).astype(np.int64)
    outstanding = 0
    i = 0

    def reap(wait_us):
        nonlocal outstanding
        got = server.collect(wait_us)
        for t in got:
            server.release(t)
        outstanding -= len(got)
        return len(got)

    while i < count or outstanding:
        if outstanding:
            reap(0)
        if i < count and Server.clock() >= arrivals[i]:
            k, v = pool[i % len(pool)]
            n = int(min(sizes[i], k.numel()))
            t = server.submit(k, v, n, int(arrivals[i]))
            if t is None:
                if not outstanding:
                    raise RuntimeError("request refused with nothing outstanding: arena or slots too small")
                reap(2000)
                continue
            outstanding += 1
            i += 1
            if i == warmup:
                while outstanding:
                    reap(2000)
                server.reset_stats()
            continue
        if i >= count:
            reap(500)
        else:
            left_us = int((arrivals[i] - Server.clock()) / 1e3)
            # a sleep or a timed wait overshoots by tens of microseconds:
            # stop short of the arrival and spin the rest
            if left_us > 200:
                if outstanding:
                    reap(min(left_us - 150, 500))
                else:
                    time.sleep(min(left_us - 150, 500) / 1e6)
    st = server.stats()
    st["gkeys_per_s"] = st["keys_sorted"] / (st["span_ms"] / 1e3) / 1e9 if st["span_ms"] > 0 else 0.0
    return st


def sweep(rates, requests: int, warmup: int, capacity: int, streams: int, seed: int = 20210708,
          verbose: bool = True, min_batch: int = 0) -> list[dict]:
    """The same seeded traces (sizes log-uniform in [2^10, 2^22], Poisson
    arrivals at each rate; rate 0 = as fast as admission allows) through a
    per-request server and a batched server."""
    from . import workloads
    desc = B.key_desc("u32", base=256, ndims=4)
    rows = []
    sizes_all = workloads.batched_sizes(requests + warmup, seed_extra=[seed])
    pool = make_pool(32, np.array([int(sizes_all.max())]), seed)  # entries long enough for every size
    for mode, name in ((B.RS_SERVE_PER_REQUEST, "per_request"), (B.RS_SERVE_BATCHED, "batched")):
        srv = Server(desc, capacity, max_slots=512, streams=streams, mode=mode, min_batch=min_batch)
        try:
            for rate in rates:
                rng = np.random.default_rng([seed, int(rate)])
                gaps = rng.exponential(1.0 / rate, requests + warmup) if rate > 0 else np.zeros(requests + warmup)
                st = run_trace(srv, pool, gaps, sizes_all, warmup=warmup)
                st.update({"mode": name, "rate": rate})
                rows.append(st)
                if verbose:
                    print(json.dumps(st), flush=True)
        finally:
            srv.close()
    return rows


def gate(rows: list[dict], ref_rate: float = 2000.0) -> dict:
    """Throughput at equal p99 latency.  Each per-request rate's p99 is a
    latency bound; within it, the best throughput each server reached over
    the sweep is compared.  `at_ref` is the bound set by the per-request
    server at ref_rate."""
    per = [r for r in rows if r["mode"] == "per_request"]
    bat = [r for r in rows if r["mode"] == "batched"]

    def best(rs, bound):
        ok = [r for r in rs if r["p99_ms"] <= bound]
        return max(ok, key=lambda r: r["gkeys_per_s"]) if ok else None

    curve = []
    for ref in sorted(per, key=lambda r: r["p99_ms"]):
        bound = ref["p99_ms"]
        b, p = best(bat, bound), best(per, bound)
        curve.append({"p99_bound_ms": round(bound, 3), "set_by_rate": ref["rate"],
                      "per_request_gkeys": round(p["gkeys_per_s"], 3) if p else None,
                      "batched_gkeys": round(b["gkeys_per_s"], 3) if b else None,
                      "batched_rate": b["rate"] if b else None})
    out = {"curve": curve}
    ref = [c for c in curve if c["set_by_rate"] == ref_rate]
    if ref:
        out["at_ref"] = ref[0]
    return out


def crossover(g: dict):
    """The smallest p99 bound of the equal-p99 curve at which the batched
    server's throughput exceeds the per-request server's, or None."""
    won = [c for c in g["curve"] if c["batched_gkeys"] is not None and c["per_request_gkeys"] is not None
           and c["batched_gkeys"] > c["per_request_gkeys"]]
    return min(won, key=lambda c: c["p99_bound_ms"]) if won else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="500,1000,2000,4000,8000,16000,32000,0")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--capacity", type=int, default=1 << 29)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--min-batch", type=int, default=0, help="batched mode: fewest queued requests batched (0 = 4)")
    ap.add_argument("--seeds", default="20210708", help="comma-separated trace seeds, one sweep each")
    a = ap.parse_args()
    summary = []
    for seed in [int(x) for x in a.seeds.split(",")]:
        rows = sweep([float(r) for r in a.rates.split(",")], a.requests, a.warmup, a.capacity, a.streams,
                     seed=seed, min_batch=a.min_batch)
        g = gate(rows)
        print(json.dumps({"seed": seed, "gate": g}), flush=True)
        summary.append({"seed": seed, "at_ref": g.get("at_ref"), "crossover": crossover(g)})
    print(json.dumps({"summary": summary}), flush=True)


if __name__ == "__main__":
    main()
