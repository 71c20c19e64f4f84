"""Seeded synthetic inputs for the sort workloads.

This module only draws random numbers. It holds none of the sort's arithmetic
(no digits, counts, scans or placement), so that the CPU oracle and the GPU
library can both be fed from it without sharing any code of the method.

Every generator uses numpy's ``Generator(PCG64)``; the draws happen in the
order written below, so a (config, seed, size) triple always yields the same
bytes for a given numpy version (recorded by ``numpy_version()``).

Workloads (seed = 20210703 + workload index):

0  ``uniform_decimal_u32``  keys uniform in [0, 10**6) as uint32, keys only;
   six base-10 digits per key (the paper's decimal count space, Section 3.1.1).
1  ``uniform_u32_pairs``    keys uniform over [0, 2**32) with the original index
   as a uint32 payload; four base-256 digits per key.
2  ``fixed_point_decimals`` lognormal(8, 2) values clipped to [0, 999999.999],
   rounded to 3 fractional digits, 30% forced integral, 10% copied from an
   earlier draw; stored as int64 scaled by 1000 (Section 3.1.2's padding to a
   common number of fractional digits), index payload.
3  ``strings16``            fixed-width 16-byte keys of lowercase a-z, length
   uniform in [1, 16], zero padded, index payload.
4  ``batched_u32``          4096 independent uint32 arrays with sizes
   log-uniform in [1024, 4194304], uniform keys, local-index payload; and a
   Poisson arrival trace for the served form.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 20210703

UNIFORM_DECIMAL_U32 = 0
UNIFORM_U32_PAIRS = 1
FIXED_POINT_DECIMALS = 2
STRINGS16 = 3
BATCHED_U32 = 4

FULL_SIZES = {
    UNIFORM_DECIMAL_U32: 1_000_000,
    UNIFORM_U32_PAIRS: 1 << 28,
    FIXED_POINT_DECIMALS: 100_000_000,
    STRINGS16: 1 << 24,
    BATCHED_U32: 4096,  # number of arrays
}

BATCH_MIN = 1024
BATCH_MAX = 4194304


def numpy_version() -> str:
    return np.__version__


def _rng(workload: int, extra=None) -> np.random.Generator:
    entropy = [SEED_BASE + workload] if extra is None else [SEED_BASE + workload, *extra]
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy)))


@dataclass
class Workload:
    """One synthetic input: keys, optional payload, and the key description."""

    name: str
    keys: np.ndarray          # uint32 [n] | int64 [n] | uint8 [n, width]
    vals: np.ndarray | None   # uint32 [n] or None (keys only)
    kind: str                 # "u32" | "u64" | "fixed_i64" | "str"
    base: int                 # radix of one dimension
    ndims: int                # number of dimensions (digits) per key
    frac_digits: int = 0      # digits after the decimal point (fixed-point only)
    str_width: int = 0        # bytes per key (strings only)

    @property
    def n(self) -> int:
        return int(self.keys.shape[0])


def uniform_decimal_u32(n: int = FULL_SIZES[UNIFORM_DECIMAL_U32], seed_extra=None) -> Workload:
    rng = _rng(UNIFORM_DECIMAL_U32, seed_extra)
    keys = rng.integers(0, 10**6, size=n, dtype=np.uint32)
    return Workload("uniform_decimal_u32", keys, None, "u32", 10, 6)


def uniform_u32_pairs(n: int = FULL_SIZES[UNIFORM_U32_PAIRS], seed_extra=None) -> Workload:
    rng = _rng(UNIFORM_U32_PAIRS, seed_extra)
    keys = rng.integers(0, 2**32, size=n, dtype=np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    return Workload("uniform_u32_pairs", keys, vals, "u32", 256, 4)


def fixed_point_decimals(n: int = FULL_SIZES[FIXED_POINT_DECIMALS], seed_extra=None) -> Workload:
    rng = _rng(FIXED_POINT_DECIMALS, seed_extra)
    x = rng.lognormal(mean=8.0, sigma=2.0, size=n)
    v = np.rint(np.clip(x, 0.0, 999999.999) * 1000.0).astype(np.int64)
    del x
    integral = rng.random(n) < 0.3
    v[integral] = (v[integral] // 1000) * 1000
    del integral
    dup = rng.random(n) < 0.1
    dup[:1] = False
    u = rng.random(n)
    idx = np.arange(n, dtype=np.int64)
    src = np.where(dup, np.floor(u * idx).astype(np.int64), idx)
    del u, dup
    # A copy takes the earlier element's final value: follow the chain of
    # sources (each strictly earlier) until it reaches an original draw.
    while True:
        nxt = src[src]
        if np.array_equal(nxt, src):
            break
        src = nxt
    v = v[src]
    del src
    vals = np.arange(n, dtype=np.uint32)
    return Workload("fixed_point_decimals", v, vals, "fixed_i64", 10, 9, frac_digits=3)


def strings16(n: int = FULL_SIZES[STRINGS16], seed_extra=None) -> Workload:
    rng = _rng(STRINGS16, seed_extra)
    lengths = rng.integers(1, 17, size=n)
    chars = rng.integers(0, 26, size=(n, 16), dtype=np.uint8) + np.uint8(ord("a"))
    chars[np.arange(16)[None, :] >= lengths[:, None]] = 0
    vals = np.arange(n, dtype=np.uint32)
    return Workload("strings16", chars, vals, "str", 27, 16, str_width=16)


def batched_sizes(count: int = FULL_SIZES[BATCHED_U32], lo: int = BATCH_MIN, hi: int = BATCH_MAX,
                  seed_extra=None) -> np.ndarray:
    """Array sizes, log-uniform in [lo, hi] (int64)."""
    rng = _rng(BATCHED_U32, seed_extra)
    s = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count)))
    return np.clip(s, lo, hi).astype(np.int64)


def batched_array(i: int, size: int, seed_extra=None) -> tuple[np.ndarray, np.ndarray]:
    """Keys and local-index payload of array ``i`` (independent stream per array)."""
    extra = [i] if seed_extra is None else [*seed_extra, i]
    rng = _rng(BATCHED_U32, [1_000_003, *extra])
    keys = rng.integers(0, 2**32, size=int(size), dtype=np.uint32)
    vals = np.arange(int(size), dtype=np.uint32)
    return keys, vals


def batched_u32(count: int = FULL_SIZES[BATCHED_U32], lo: int = BATCH_MIN, hi: int = BATCH_MAX,
                seed_extra=None):
    """Concatenated arrays plus segment offsets (uint64, count + 1 entries)."""
    sizes = batched_sizes(count, lo, hi, seed_extra)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes).astype(np.uint64)
    total = int(offsets[-1])
    keys = np.empty(total, dtype=np.uint32)
    vals = np.empty(total, dtype=np.uint32)
    for i in range(count):
        a, b = int(offsets[i]), int(offsets[i + 1])
        keys[a:b], vals[a:b] = batched_array(i, b - a, seed_extra)
    return keys, vals, offsets


def arrival_trace(count: int, rate_per_s: float, lo: int = BATCH_MIN, hi: int = BATCH_MAX,
                  seed_extra=None) -> tuple[np.ndarray, np.ndarray]:
    """Poisson arrivals: (arrival times in seconds from 0, request sizes)."""
    rng = _rng(BATCHED_U32, [2_000_003, *(seed_extra or [])])
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    s = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count)))
    return t, np.clip(s, lo, hi).astype(np.int64)


def paper_decimal_case(n: int, hi: int, frac_digits: int, seed: int = 0) -> np.ndarray:
    """Section 6's data shape: values in [1, hi) with ``frac_digits`` decimals,
    as int64 fixed-point (value * 10**frac_digits)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 6, hi, frac_digits, seed])))
    scale = 10**frac_digits
    return rng.integers(1 * scale, hi * scale, size=n, dtype=np.int64)


def by_index(workload: int, n: int | None = None, seed_extra=None) -> Workload:
    makers = {
        UNIFORM_DECIMAL_U32: uniform_decimal_u32,
        UNIFORM_U32_PAIRS: uniform_u32_pairs,
        FIXED_POINT_DECIMALS: fixed_point_decimals,
        STRINGS16: strings16,
    }
    fn = makers[workload]
    return fn(FULL_SIZES[workload] if n is None else n, seed_extra=seed_extra)
