"""Base-27 strings of 16 symbols from 2^21 keys (the prescanned passes): the passes over the four
leading symbols, then every bucket of equal leading symbols sorted on its own
by the other twelve (waves for buckets of at most 64 keys, buckets of equal
keys left as they are, the batched passes for longer buckets whose keys
differ).  Every case is compared with the oracle element by element,
ascending and descending, with and without values."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import workloads
from tests.gpu_helpers import assert_same, gpu_sort, oracle_sort

pytestmark = pytest.mark.gpu

N = (1 << 21) + 17


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    B.rs_tuning_clear()


def _strings(case, n=N):
    rng = np.random.default_rng(20210703 + len(case))
    if case == "uniform":
        return workloads.strings16(n, seed_extra=(7,)).keys
    letters = lambda shape: (rng.integers(0, 26, shape, dtype=np.uint8) + np.uint8(ord("a")))  # noqa: E731
    k = np.zeros((n, 16), np.uint8)
    if case == "one_prefix":
        # every key starts with "abcd": one bucket of n distinct keys
        k[:, :4] = np.frombuffer(b"abcd", np.uint8)
        k[:, 4:] = letters((n, 12))
        cut = rng.integers(5, 17, n)
        k[np.arange(16)[None, :] >= cut[:, None]] = 0
    elif case == "mixed_buckets":
        # 300 prefixes of 1..8000 keys each with random tails, plus short
        # duplicated keys (long buckets of equal keys)
        sizes = rng.integers(1, 8000, 300)
        pref = letters((300, 4))
        rows = np.repeat(np.arange(300), sizes)[:n]
        k[: rows.shape[0], :4] = pref[rows]
        k[: rows.shape[0], 4:] = letters((rows.shape[0], 12))
        cut = rng.integers(4, 17, rows.shape[0])
        k[: rows.shape[0]][np.arange(16)[None, :] >= cut[:, None]] = 0
        rest = n - rows.shape[0]
        if rest > 0:
            short = letters((rest, 2))
            short[:, 1] = np.where(rng.random(rest) < 0.5, short[:, 1], 0)
            k[rows.shape[0]:, :2] = short
        rng.shuffle(k)
    elif case == "lengths_up_to_4":
        # only keys of at most four symbols: every bucket holds equal keys
        k[:, :4] = letters((n, 4))
        cut = rng.integers(1, 5, n)
        k[np.arange(16)[None, :] >= cut[:, None]] = 0
    elif case == "near_64":
        # buckets of 60..70 keys around the one-wave limit
        nb = n // 60 + 1
        sizes = rng.integers(60, 71, nb)
        rows = np.repeat(np.arange(nb), sizes)[:n]
        pref = letters((nb, 4))
        k[:, :4] = pref[rows]
        k[:, 4:] = letters((n, 12))
        rng.shuffle(k)
    elif case == "change_points":
        # buckets of 2..300 keys, each one tail repeated and then another
        # from a change point on, so that a bucket's only differing
        # neighbours sit at the change point; in the ordered array the
        # change points fall where a wave's 64-key step or its range of the
        # count begins (n is 384 × 8192: ranges of 384 keys when 8192 waves
        # count), which the count kernel sees through the key carried from
        # the step or range before
        sizes = rng.integers(2, 301, n // 2)
        sizes = sizes[: np.searchsorted(np.cumsum(sizes), n) + 1]
        sizes[-1] -= int(sizes.sum()) - n
        nb = sizes.shape[0]
        cells = np.sort(rng.choice(26 ** 4, nb, replace=False))
        pref = np.stack([cells // 26 ** (3 - j) % 26 for j in range(4)], axis=1).astype(np.uint8) + np.uint8(97)
        starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        step = np.where(np.arange(nb) % 3 == 0, 384, 64)
        at = (starts // step + 1) * step  # first such boundary after the bucket's start
        inside = at < starts + sizes
        change = np.where(inside, at - starts, rng.integers(1, np.maximum(sizes, 2)))
        change = np.minimum(change, sizes - 1)
        tails = letters((nb, 2, 12))
        rows = np.repeat(np.arange(nb), sizes)
        second = (np.arange(n) - starts[rows]) >= change[rows]
        k[:, :4] = pref[rows]
        k[:, 4:] = tails[rows, second.astype(np.int64)]
        # buckets in shuffled order, each keeping its own order
        order = rng.permutation(nb)
        k = np.concatenate([k[starts[b]: starts[b] + sizes[b]] for b in order])
    return k


@pytest.mark.parametrize("case", ["uniform", "one_prefix", "mixed_buckets", "lengths_up_to_4", "near_64",
                                  "change_points"])
@pytest.mark.parametrize("descending", [False, True])
def test_bucketed_strings_pairs(case, descending):
    keys = _strings(case, 384 * 8192) if case == "change_points" else _strings(case)
    n = keys.shape[0]
    vals = np.arange(n, dtype=np.uint32)
    _say(f"bucketed strings {case} desc={descending} n={n}")
    d = B.key_desc("str", base=27, ndims=16, descending=descending)
    assert B.rs_plan_inspect(d, n, True).form == B.RS_FORM_PRESCANNED
    gk, gv = gpu_sort(keys, vals, "str", 27, 16, descending=descending)
    ok, ov = oracle_sort(keys, vals, "str", 27, 16, descending=descending)
    assert_same(gk, gv, ok, ov, f"{case} desc={descending}")


@pytest.mark.parametrize("case", ["uniform", "mixed_buckets"])
def test_bucketed_strings_keys_only_in_place(case):
    keys = _strings(case)
    _say(f"bucketed strings keys only in place {case}")
    gk, _ = gpu_sort(keys, None, "str", 27, 16, in_place=True)
    ok, _ = oracle_sort(keys, None, "str", 27, 16)
    assert_same(gk, None, ok, None, case)


def test_bucketed_strings_graph_replay_equals_eager():
    """Under capture the form cannot wait for the long-bucket count, so the
    captured sequence runs all eight passes; its replays equal the eager
    (bucketed) result."""
    import torch
    from paper_2107_01391_amd import api
    keys = _strings("mixed_buckets")
    n = keys.shape[0]
    vals = np.arange(n, dtype=np.uint32)
    d = B.key_desc("str", base=27, ndims=16)
    kd, vd = api.to_device(keys), api.to_device(vals)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    tmp = api.empty_device(B.rs_temp_bytes(d, n, True))
    g = B.rs_graph_sort(d, kd, ko, vd, vo, n, tmp, tmp.numel())
    eager_k, eager_v = gpu_sort(keys, vals, "str", 27, 16)
    for rep in range(3):
        ko.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(api.to_host(ko, np.uint8, (n, 16)), eager_k), f"replay {rep}"
        assert np.array_equal(api.to_host(vo, np.uint32, (n,)), eager_v), f"replay {rep}"
    g.close()
