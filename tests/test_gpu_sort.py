"""Parity of the HIP path with the CPU oracle, element by element, on seeded
inputs that span several tiles and a ragged tail, plus the edge cases."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import workloads
from tests.gpu_helpers import assert_same, gpu_sort, oracle_sort

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()  # raises when librs.so was not built: no fallback


TILE_U32 = 4096  # keys per tile of the 32/64-bit kernels
TILE_STR = 2048


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, TILE_U32 - 1, TILE_U32, TILE_U32 + 1, 3 * TILE_U32 + 17, 100_003,
                               1 << 20])
def test_u32_pairs_base256(n):
    _say(f"u32 pairs base 256 n={n}")
    w = workloads.uniform_u32_pairs(n)
    gk, gv = gpu_sort(w.keys, w.vals, "u32", 256, 4)
    ok, ov = oracle_sort(w.keys, w.vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov, f"n={n}")


def test_empty_is_noop():
    import torch
    d = B.key_desc("u32")
    B.rs_sort_pairs(d, 0, 0, 0, 0, 0, 0, 0)
    B.rs_sort_keys(d, 0, 0, 0, 0, 0)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 1000, 65_537, 1_000_000])
def test_decimal_keys_literal(n):
    """Keys only on a 10^6-cell space: count, scan, emit rebuilt keys."""
    _say(f"decimal keys literal n={n}")
    w = workloads.uniform_decimal_u32(n)
    gk, _ = gpu_sort(w.keys, None, "u32", 10, 6)
    ok, _ = oracle_sort(w.keys, None, "u32", 10, 6, groups=[6])
    assert_same(gk, None, ok, None, f"n={n}")


@pytest.mark.parametrize("case", ["clustered", "two_rows", "extremes", "one_key", "one_dim", "u64_rows"])
def test_literal_traverse_maps(case):
    """Keys only on small spaces, where the count kernel also builds the
    traverse maps (each row's occupied range) and the scan and emit skip
    what lies outside: sparse and clustered occupancy, the first and last
    cells, a single key, a one-dimensional space (one row)."""
    _say(f"literal traverse maps {case}")
    rng = np.random.default_rng(len(case))
    kind, base, ndims, dt = "u32", 16, 6, np.uint32
    if case == "clustered":  # 2^22 keys inside 1/256 of a 2^24-cell space
        keys = rng.integers(0x350000, 0x360000, 1 << 22, dtype=np.uint32)
    elif case == "two_rows":  # rows 2 and 13, narrow columns
        a = rng.integers(2 * 2**20 + 1000, 2 * 2**20 + 5000, 300_000, dtype=np.uint32)
        b = rng.integers(13 * 2**20 + 777, 13 * 2**20 + 9000, 300_000, dtype=np.uint32)
        keys = np.concatenate([a, b])
        rng.shuffle(keys)
    elif case == "extremes":
        keys = rng.choice(np.array([0, 1, 2**24 - 2, 2**24 - 1], np.uint32), 200_000)
    elif case == "one_key":
        keys = np.full(100_000, 2**23 + 12345, np.uint32)
    elif case == "one_dim":
        base, ndims = 60_000, 1
        keys = rng.integers(1000, 2000, 70_000, dtype=np.uint32)
    else:
        kind, base, ndims, dt = "u64", 10, 6, np.uint64
        keys = rng.integers(400_000, 420_000, 250_000, dtype=np.uint64)
    gk, _ = gpu_sort(keys.astype(dt), None, kind, base, ndims)
    assert np.array_equal(gk, np.sort(keys.astype(dt)))
    if keys.shape[0] <= 400_000:
        ok, _ = oracle_sort(keys.astype(dt), None, kind, base, ndims)
        assert_same(gk, None, ok, None)


@pytest.mark.parametrize("n", [5000, 300_001])
def test_decimal_pairs_base10(n):
    _say(f"decimal pairs base 10 n={n}")
    w = workloads.uniform_decimal_u32(n)
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort(w.keys, vals, "u32", 10, 6)
    ok, ov = oracle_sort(w.keys, vals, "u32", 10, 6)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("n", [4097, 200_003])
def test_fixed_point_pairs(n):
    _say(f"fixed point pairs n={n}")
    w = workloads.fixed_point_decimals(n)
    gk, gv = gpu_sort(w.keys, w.vals, "fixed_i64", 10, 9, frac_digits=3)
    ok, ov = oracle_sort(w.keys, w.vals, "fixed_i64", 10, 9)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("n", [1, 2047, 2049, 50_003])
def test_strings_pairs(n):
    _say(f"strings pairs n={n}")
    w = workloads.strings16(n)
    gk, gv = gpu_sort(w.keys, w.vals, "str", 27, 16)
    ok, ov = oracle_sort(w.keys, w.vals, "str", 27, 16)
    assert_same(gk, gv, ok, ov)


def test_strings_keys_only():
    _say("strings keys only")
    w = workloads.strings16(30_001)
    gk, _ = gpu_sort(w.keys, None, "str", 27, 16)
    ok, _ = oracle_sort(w.keys, None, "str", 27, 16)
    assert_same(gk, None, ok, None)


@pytest.mark.parametrize("base,ndims,prescan", [(1000, 3, False), (1000, 3, True), (37, 6, True)])
def test_other_bases(monkeypatch, base, ndims, prescan):
    """Bases above the default pass width (1000 cells, the 10-bit kernels)
    and an odd base with two-digit passes (37^2 = 1369 > 256: one digit)."""
    monkeypatch.setenv("RS_PRESCAN_MIN_N", "1" if prescan else str(1 << 40))
    _say(f"base {base} ndims {ndims} prescan={prescan}")
    rng = np.random.default_rng(base)
    n = 250_003
    keys = rng.integers(0, base ** ndims, n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "u32", base, ndims)
    ok, ov = oracle_sort(keys, vals, "u32", base, ndims)
    assert_same(gk, gv, ok, ov)


def test_u64_pairs():
    _say("u64 pairs")
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 2**64, 100_003, dtype=np.uint64)
    keys[::5] = keys[7]
    vals = np.arange(keys.shape[0], dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "u64", 256, 8)
    ok, ov = oracle_sort(keys, vals, "u64", 256, 8)
    assert_same(gk, gv, ok, ov)


def test_u32_keys_only_passes():
    _say("u32 keys only, grouped passes")
    w = workloads.uniform_u32_pairs(77_777)
    gk, _ = gpu_sort(w.keys, None, "u32", 256, 4)
    ok, _ = oracle_sort(w.keys, None, "u32", 256, 4)
    assert_same(gk, None, ok, None)


@pytest.mark.parametrize("distinct", [1, 2, 3, 17])
def test_skewed_hot_cells(distinct):
    """All keys in a handful of cells: the single-cell hot spot of the count."""
    _say(f"skewed distinct={distinct}")
    rng = np.random.default_rng(distinct)
    pool = rng.integers(0, 2**32, distinct, dtype=np.uint32)
    keys = pool[rng.integers(0, distinct, 150_001)]
    vals = np.arange(keys.shape[0], dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "u32", 256, 4)
    ok, ov = oracle_sort(keys, vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("kind,base,ndims", [("u32", 256, 4), ("fixed_i64", 10, 9)])
def test_in_place(kind, base, ndims):
    """keys_out == keys_in: even (4) and odd (3) pass counts."""
    _say(f"in place {kind}")
    if kind == "u32":
        w = workloads.uniform_u32_pairs(123_457)
    else:
        w = workloads.fixed_point_decimals(123_457)
    gk, gv = gpu_sort(w.keys, w.vals, kind, base, ndims, in_place=True)
    ok, ov = oracle_sort(w.keys, w.vals, kind, base, ndims)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("prescan", [False, True])
@pytest.mark.parametrize("kind,base,ndims,elem", [("u32", 256, 4, 1), ("u32", 256, 4, 3), ("u64", 256, 8, 1)])
def test_slices_not_16_byte_aligned(monkeypatch, prescan, kind, base, ndims, elem):
    """Arrays that start `elem` keys into a buffer: the 128-bit count loads
    give way to one key per load."""
    import torch
    monkeypatch.setenv("RS_PRESCAN_MIN_N", "1" if prescan else str(1 << 40))
    _say(f"slice at +{elem} {kind} prescan={prescan}")
    n = 3 * TILE_U32 + 77
    rng = np.random.default_rng(5 + elem)
    dt = np.uint32 if kind == "u32" else np.uint64
    keys = rng.integers(0, np.iinfo(dt).max, n, dtype=dt, endpoint=True)
    vals = np.arange(n, dtype=np.uint32)
    kb = keys.itemsize
    kbuf = torch.zeros((n + elem) * kb, dtype=torch.uint8, device="cuda")
    kbuf[elem * kb:].copy_(torch.from_numpy(keys.view(np.uint8)).cuda())
    vbuf = torch.zeros((n + 1) * 4, dtype=torch.uint8, device="cuda")
    vbuf[4:].copy_(torch.from_numpy(vals.view(np.uint8)).cuda())
    kout = torch.zeros((n + elem) * kb, dtype=torch.uint8, device="cuda")
    vout = torch.zeros((n + 1) * 4, dtype=torch.uint8, device="cuda")
    d = B.key_desc(kind, base=base, ndims=ndims)
    tmp = torch.empty(B.rs_temp_bytes(d, n, True), dtype=torch.uint8, device="cuda")
    B.rs_sort_pairs(d, kbuf[elem * kb:], kout[elem * kb:], vbuf[4:], vout[4:], n, tmp, tmp.numel())
    torch.cuda.synchronize()
    gk = kout[elem * kb:].cpu().numpy().view(dt)
    gv = vout[4:].cpu().numpy().view(np.uint32)
    ok, ov = oracle_sort(keys, vals, kind, base, ndims)
    assert_same(gk, gv, ok, ov)
    assert not kout[: elem * kb].any() and not vout[:4].any(), "wrote before the slice"


def test_deterministic_repeat():
    _say("determinism")
    w = workloads.uniform_u32_pairs(500_000)
    a = gpu_sort(w.keys, w.vals, "u32", 256, 4)
    b = gpu_sort(w.keys, w.vals, "u32", 256, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_validate_rejects_out_of_space_keys():
    _say("validate")
    keys = np.array([5, 999_999, 1_000_000, 3], np.uint32)
    with pytest.raises(B.RSError) as e:
        gpu_sort(keys, None, "u32", 10, 6, validate=True)
    assert e.value.status == 3
    keys = np.array([[ord("a")] + [0] * 14 + [ord("A")]], np.uint8)
    with pytest.raises(B.RSError) as e:
        gpu_sort(keys, np.zeros(1, np.uint32), "str", 27, 16, validate=True)
    assert e.value.status == 3
    ok_keys = np.array([5, 999_999, 3], np.uint32)
    gk, _ = gpu_sort(ok_keys, None, "u32", 10, 6, validate=True)
    assert gk.tolist() == [3, 5, 999_999]


# ------------------------------------------------------- prescanned passes
# Large single arrays run every pass as per-tile counts, one flat scan and a
# scatter whose offsets come from the scanned table; small ones chain their
# tiles by look-back.  The switch point is lowered here so that ragged,
# skewed and in-place cases stay small; setting it above n forces the chain.

@pytest.fixture()
def prescanned(monkeypatch):
    monkeypatch.setenv("RS_PRESCAN_MIN_N", "1")
    yield


@pytest.fixture()
def chained(monkeypatch):
    monkeypatch.setenv("RS_PRESCAN_MIN_N", str(1 << 40))
    yield


@pytest.mark.parametrize("n", [1, 2, 63, TILE_U32 - 1, TILE_U32, TILE_U32 + 1, 8 * TILE_U32 + 1, 70_001, 1 << 20])
def test_prescanned_u32_pairs(prescanned, n):
    _say(f"prescanned u32 pairs n={n}")
    w = workloads.uniform_u32_pairs(n)
    gk, gv = gpu_sort(w.keys, w.vals, "u32", 256, 4)
    ok, ov = oracle_sort(w.keys, w.vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov, f"n={n}")


def test_chained_large(chained):
    _say("chained u32 pairs n=3M")
    w = workloads.uniform_u32_pairs(3_000_017)
    gk, gv = gpu_sort(w.keys, w.vals, "u32", 256, 4)
    ok, ov = oracle_sort(w.keys, w.vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov)


def test_prescanned_keys_only_and_in_place(prescanned):
    _say("prescanned keys only, in place")
    w = workloads.uniform_u32_pairs(99_999)
    gk, _ = gpu_sort(w.keys, None, "u32", 256, 4)
    ok, _ = oracle_sort(w.keys, None, "u32", 256, 4)
    assert_same(gk, None, ok, None)
    gk, gv = gpu_sort(w.keys, w.vals, "u32", 256, 4, in_place=True)
    ok, ov = oracle_sort(w.keys, w.vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov)


def test_prescanned_fixed_point_skewed(prescanned):
    """Fixed point: 1000-cell groups, most keys in a few cells (the lognormal
    skew), three passes: odd, so in place starts from a copy."""
    _say("prescanned fixed point")
    w = workloads.fixed_point_decimals(300_007)
    gk, gv = gpu_sort(w.keys, w.vals, "fixed_i64", 10, 9, frac_digits=3)
    ok, ov = oracle_sort(w.keys, w.vals, "fixed_i64", 10, 9)
    assert_same(gk, gv, ok, ov)
    gk, gv = gpu_sort(w.keys, w.vals, "fixed_i64", 10, 9, in_place=True)
    assert_same(gk, gv, ok, ov, "in place, odd pass count")


def test_prescanned_strings_and_u64(prescanned):
    _say("prescanned strings")
    w = workloads.strings16(60_001)
    gk, gv = gpu_sort(w.keys, w.vals, "str", 27, 16)
    ok, ov = oracle_sort(w.keys, w.vals, "str", 27, 16)
    assert_same(gk, gv, ok, ov)
    _say("prescanned u64")
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 2**64, 50_001, dtype=np.uint64)
    vals = np.arange(keys.shape[0], dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "u64", 256, 8)
    ok, ov = oracle_sort(keys, vals, "u64", 256, 8)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("distinct", [1, 5])
def test_prescanned_hot_cells(prescanned, distinct):
    _say(f"prescanned skewed distinct={distinct}")
    rng = np.random.default_rng(100 + distinct)
    pool = rng.integers(0, 2**32, distinct, dtype=np.uint32)
    keys = pool[rng.integers(0, distinct, 200_003)]
    vals = np.arange(keys.shape[0], dtype=np.uint32)
    gk, gv = gpu_sort(keys, vals, "u32", 256, 4)
    ok, ov = oracle_sort(keys, vals, "u32", 256, 4)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("kind,n", [("u32", 1), ("u32", 8191), ("u32", 8192), ("u32", 8193), ("u32", 5 * 8192 + 3),
                                    ("u32", 1 << 20), ("u64", 70_001), ("fixed_i64", 100_003)])
def test_prescanned_wide_tiles(prescanned, monkeypatch, kind, n):
    """512-thread tiles (8192 keys) for 4- and 8-byte keys."""
    monkeypatch.setenv("RS_TILE_BLOCK", "512")
    _say(f"prescanned wide tiles {kind} n={n}")
    if kind == "u32":
        w = workloads.uniform_u32_pairs(n)
        args = ("u32", 256, 4)
        keys, vals = w.keys, w.vals
    elif kind == "u64":
        rng = np.random.default_rng(9)
        keys = rng.integers(0, 2**64, n, dtype=np.uint64)
        vals = np.arange(n, dtype=np.uint32)
        args = ("u64", 256, 8)
    else:
        w = workloads.fixed_point_decimals(n)
        keys, vals = w.keys, w.vals
        args = ("fixed_i64", 10, 9)
    gk, gv = gpu_sort(keys, vals, *args)
    ok, ov = oracle_sort(keys, vals, *args)
    assert_same(gk, gv, ok, ov, f"n={n}")
    gk, gv = gpu_sort(keys, vals, *args, in_place=True)
    assert_same(gk, gv, ok, ov, f"in place n={n}")
    gk, _ = gpu_sort(keys, None, *args)
    assert_same(gk, None, ok, None, f"keys only n={n}")


@pytest.mark.parametrize("tile_block", [256, 512])
@pytest.mark.parametrize("base,ndims,bits", [(16, 8, 4), (2, 32, 11), (4, 16, 10)])
def test_prescanned_digit_widths(prescanned, monkeypatch, tile_block, base, ndims, bits):
    """Other pass widths on power-of-two bases: 8 passes of 16 cells; passes
    of 2048, 2048 and 1024 cells (2048-cell passes keep 256-thread tiles
    whatever the tuning asks); 1024-cell passes."""
    monkeypatch.setenv("RS_DIGIT_BITS", str(bits))
    monkeypatch.setenv("RS_TILE_BLOCK", str(tile_block))
    _say(f"prescanned base {base} digit bits {bits} tile block {tile_block}")
    w = workloads.uniform_u32_pairs(123_457)
    gk, gv = gpu_sort(w.keys, w.vals, "u32", base, ndims)
    ok, ov = oracle_sort(w.keys, w.vals, "u32", base, ndims)
    assert_same(gk, gv, ok, ov)


@pytest.mark.parametrize("n", [100_003, 3_500_001], ids=["chained", "prescanned"])
@pytest.mark.parametrize("pattern", ["sorted", "reverse", "all_equal", "two_values"])
def test_ordered_and_degenerate_inputs(pattern, n):
    """Inputs whose stable sort is known in closed form: already sorted
    (identity), reverse sorted with distinct keys (reversal), all keys equal
    (identity: every tie keeps input order), two alternating values (evens
    then odds).  Every key of a tile in one cell is the worst case of the
    count tables' atomics."""
    _say(f"ordered input {pattern} n={n}")
    idx = np.arange(n, dtype=np.uint64)
    if pattern == "sorted":
        keys = (idx * 61).astype(np.uint32)
        want = idx
    elif pattern == "reverse":
        keys = ((n - idx) * 61).astype(np.uint32)
        want = idx[::-1]
    elif pattern == "all_equal":
        keys = np.full(n, 0xDEADBEEF, np.uint32)
        want = idx
    else:
        keys = np.where(idx % 2 == 0, 7, 0x7000000).astype(np.uint32)
        want = np.concatenate([idx[0::2], idx[1::2]])
    vals = idx.astype(np.uint32)
    gk, gv = gpu_sort(keys, vals, "u32", 256, 4)
    assert np.array_equal(gv, want.astype(np.uint32)), pattern
    assert np.array_equal(gk, keys[want.astype(np.int64)]), pattern


@pytest.mark.parametrize("kind,base,ndims", [("u64", 256, 4), ("u64", 10, 9), ("fixed_i64", 10, 9)],
                         ids=["u64-b256-even", "u64-b10-odd", "fixed-odd"])
@pytest.mark.parametrize("form", ["pairs", "keys_in_place", "pairs_in_place_desc"])
def test_narrowed_eight_byte_keys(kind, base, ndims, form):
    """8-byte keys whose space fits 32 bits, at a size that takes the
    prescanned passes: narrowed to 32-bit words for the passes and widened
    at the end (even and odd pass counts, in place, descending)."""
    n = 3_300_007
    _say(f"narrowed {kind} base {base} ndims {ndims} {form} n={n}")
    rng = np.random.default_rng(n + ndims)
    space = base ** ndims
    keys = rng.integers(0, space, n, dtype=np.int64 if kind == "fixed_i64" else np.uint64)
    keys[::7] = keys[3]  # ties
    keys[0], keys[1] = 0, space - 1
    desc = form.endswith("desc")
    vals = None if form.startswith("keys") else rng.permutation(n).astype(np.uint32)
    gk, gv = gpu_sort(keys, vals, kind, base, ndims, in_place="in_place" in form, descending=desc)
    ok, ov = oracle_sort(keys, vals, kind, base, ndims, descending=desc)
    assert_same(gk, gv, ok, ov, f"{kind} {form}")
