"""Pins of the CPU oracle against what the paper and plain mathematics fix.

Every ``pin_*`` function raises AssertionError (or OracleError) when the
oracle is wrong.  ``test_mutants_are_caught`` builds edited copies of the
oracle's C source -- each with one plausible mistake (a wrong bound, index,
comparison or order) -- and checks that at least one pin rejects every one,
so the pins are not just the oracle agreeing with itself.
"""
from __future__ import annotations

import itertools
import json
import os
from decimal import Decimal

import numpy as np
import pytest

import oracle
from paper_2107_01391_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _fixed(decimals, frac_digits):
    """Exact decimal strings -> int64 fixed point (value * 10**frac)."""
    return np.array([int(Decimal(s).scaleb(frac_digits)) for s in decimals], dtype=np.int64)


def _stable_order(keys):
    """Brute-force stable order: input indices sorted by (key, index)."""
    return sorted(range(len(keys)), key=lambda i: (keys[i], i))


# ------------------------------------------------------------------ pins

def pin_worked_example_output():
    ex = _golden("worked_example.json")["worked_example"]
    keys = _fixed(ex["input"], ex["frac_digits"])
    want = _fixed(ex["sorted"], ex["frac_digits"])
    vals = np.arange(len(keys), dtype=np.uint32)
    ko, vo, st = oracle.sort(keys, vals, kind="fixed_i64", base=ex["base"], ndims=ex["ndims"])
    assert ko.tolist() == want.tolist()
    assert vo.tolist() == ex["stable_payload"]
    assert st.cells_visited == ex["k"]
    ko2, _, st2 = oracle.sort(keys, None, kind="fixed_i64", base=ex["base"], ndims=ex["ndims"])
    assert ko2.tolist() == want.tolist()
    assert st2.cells_visited == ex["k"]


def pin_worked_example_hashing_state():
    ex = _golden("worked_example.json")["worked_example"]
    keys = _fixed(ex["input"], ex["frac_digits"])
    h = oracle.hash_level(keys, kind="fixed_i64", base=10, ndims=2)
    S = np.zeros((10, 10), np.uint64)
    for r, c, cnt in ex["S_cells"]:
        S[r, c] = cnt
    assert np.array_equal(h["S"], S)
    assert h["hmax"][:, 0].tolist() == ex["H_Max"]
    assert [[int(f), int(m)] for f, m in zip(h["hmin_flag"][:, 0], h["hmin"][:, 0])] == ex["H_Min"]
    assert h["hmin"][4, 0] == ex["row4_min"] and h["hmax"][4, 0] == ex["row4_max"]
    assert h["k"] == ex["k"]
    # I_Hash at termination: every element is mapped (Section 4.1)
    assert int(h["S"].sum()) == len(keys)
    # the walk hands out positions as a running sum in lexicographic order
    pos = 0
    for cell in range(100):
        if S.flat[cell]:
            assert h["start"].flat[cell] == pos
            pos += int(S.flat[cell])


def pin_padding_example():
    ex = _golden("worked_example.json")["padding_example"]
    a = _fixed(ex["input"], ex["frac_digits"])
    b = _fixed(ex["padded"], ex["frac_digits"])
    assert a.tolist() == b.tolist() == [101, 210, 100]
    ko, _, _ = oracle.sort(a, None, kind="fixed_i64", base=10, ndims=3)
    assert ko.tolist() == [100, 101, 210]


def pin_table3_shapes():
    t3 = _golden("table3.json")
    for row in t3["rows"]:
        scale = 10 ** row["cd"]
        n = oracle.dims_for(row["hi"] * scale, 10)
        assert [10] * n == row["count_array"], row
        keys = workloads.paper_decimal_case(200, row["hi"], row["cd"], seed=1)
        h = oracle.hash_level(keys, kind="fixed_i64", base=10, ndims=n)
        assert list(h["S"].shape) == row["count_array"]
        if n == 1:
            assert [2 * h["hmin"].size] == row["h_min"] and [h["hmax"].size] == row["h_max"]
        else:
            assert [h["hmin"].shape[0]] + [2] * h["hmin"].shape[1] == row["h_min"]
            assert [h["hmax"].shape[0]] + [1] * h["hmax"].shape[1] == row["h_max"]


_TINY_CASES = [
    # kind, base, ndims, groups list, alphabet of keys
    ("u32", 10, 2, [[2], [1, 1]], [0, 7, 70, 77, 99]),
    ("u32", 256, 4, [[1, 3], [1, 1, 1, 1], [2, 2]], [0, 1, 256, 65536, 2**32 - 1]),
    ("u64", 256, 8, [[1, 1, 1, 1, 1, 1, 1, 1], [2, 2, 2, 2]], [0, 2**63, 2**40 + 3, 5, 2**64 - 1]),
    ("fixed_i64", 10, 3, [[3], [1, 2], [2, 1]], [100, 101, 210, 9, 990]),
]


def pin_brute_force_tiny():
    """Every sequence of length <= 5 over a 3-key alphabet, all kinds and groupings."""
    for kind, base, ndims, groupings, alphabet in _TINY_CASES:
        for alpha in itertools.combinations(alphabet, 3):
            for length in range(0, 6):
                for seq in itertools.product(alpha, repeat=length):
                    dt = {"u32": np.uint32, "u64": np.uint64, "fixed_i64": np.int64}[kind]
                    keys = np.array(seq, dtype=dt)
                    vals = np.arange(length, dtype=np.uint32)
                    order = _stable_order([int(k) for k in seq])
                    for groups in groupings:
                        ko, vo, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups)
                        assert vo.tolist() == order, (kind, groups, seq)
                        assert ko.tolist() == [int(seq[i]) for i in order]
                        ko2, _, _ = oracle.sort(keys, None, kind=kind, base=base, ndims=ndims, groups=groups)
                        assert ko2.tolist() == sorted(int(s) for s in seq)


def _str_rows(words, width):
    out = np.zeros((len(words), width), np.uint8)
    for i, w in enumerate(words):
        b = w.encode()
        out[i, :len(b)] = np.frombuffer(b, np.uint8)
    return out


def pin_brute_force_strings():
    """Strings follow memcmp order of the zero-padded rows (pad sorts first)."""
    words = ["", "a", "ab", "b", "ba", "zz", "aab"]
    for alpha in itertools.combinations(words, 3):
        for length in range(0, 6):
            for seq in itertools.product(alpha, repeat=length):
                keys = _str_rows(seq, 3)
                rows = [bytes(r) for r in keys]
                order = _stable_order(rows)
                vals = np.arange(length, dtype=np.uint32)
                for groups in ([3], [1, 2], [1, 1, 1]):
                    ko, vo, _ = oracle.sort(keys, vals, kind="str", base=27, ndims=3, groups=groups)
                    assert vo.tolist() == order, (seq, groups)
                    assert [bytes(r) for r in ko] == [rows[i] for i in order]
                    ko2, _, _ = oracle.sort(keys, None, kind="str", base=27, ndims=3, groups=groups)
                    assert [bytes(r) for r in ko2] == sorted(rows)


def pin_medium_vs_library_stable_sort():
    """Larger seeded inputs against numpy's stable argsort (a library routine)."""
    rng = np.random.default_rng(7)
    cases = []
    k = rng.integers(0, 10**6, 20000, dtype=np.uint32)
    cases.append((k, "u32", 10, 6, [[6], [3, 3], [2, 2, 2], [1, 5]]))
    k = rng.integers(0, 2**32, 20000, dtype=np.uint32)
    k[::7] = k[3]  # heavy duplicates
    cases.append((k, "u32", 256, 4, [[1, 3], [1, 1, 1, 1], [2, 2]]))
    k = rng.integers(0, 2**64, 5000, dtype=np.uint64)
    cases.append((k, "u64", 256, 8, [[1] * 8]))
    k = workloads.fixed_point_decimals(20000).keys
    cases.append((k, "fixed_i64", 10, 9, [[3, 6], [3, 3, 3]]))
    for keys, kind, base, ndims, groupings in cases:
        want = np.argsort(keys, kind="stable")
        vals = np.arange(keys.shape[0], dtype=np.uint32)
        for groups in groupings:
            ko, vo, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups)
            assert np.array_equal(vo, want.astype(np.uint32)), (kind, groups)
            assert np.array_equal(ko, keys[want])
    w = workloads.strings16(3000)
    rows = [bytes(r) for r in w.keys]
    order = sorted(range(len(rows)), key=lambda i: (rows[i], i))
    ko, vo, _ = oracle.sort(w.keys, w.vals, kind="str", base=27, ndims=16, groups=[2] * 8)
    assert vo.tolist() == order
    ko, vo, _ = oracle.sort(w.keys, w.vals, kind="str", base=27, ndims=16, groups=[4] * 4)
    assert vo.tolist() == order


def pin_literal_walk_cost():
    """k of one literal level: a dense 1-D space walks max-min+1 cells; a
    2-D space walks, per touched row, its column range (Section 5)."""
    keys = np.array([5, 2, 9, 2], np.uint32)
    _, _, st = oracle.sort(keys, None, kind="u32", base=10, ndims=1)
    assert st.cells_visited == 9 - 2 + 1
    keys = np.array([12, 18, 45, 41, 44], np.uint32)  # rows 1 (cols 2..8), 4 (cols 1..5)
    _, _, st = oracle.sort(keys, None, kind="u32", base=10, ndims=2)
    assert st.cells_visited == 7 + 5
    # all keys in one cell: one cell walked (best case iii of Section 5)
    _, _, st = oracle.sort(np.full(50, 31, np.uint32), None, kind="u32", base=10, ndims=2)
    assert st.cells_visited == 1


_SIGNED_DESC_CASES = [
    # kind, base, ndims, groups list, alphabet, descending
    ("i32", 256, 4, [[1, 3], [1, 1, 1, 1]], [-2**31, -1, 0, 1, 2**31 - 1, -300], False),
    ("i32", 10, 10, [[2] * 5, [4, 6]], [-2**31, -7, 0, 9, 2**31 - 1], False),
    ("i64", 256, 8, [[1] * 8, [2, 2, 2, 2]], [-2**63, -2**40, -1, 0, 3, 2**63 - 1], False),
    ("i64", 16, 16, [[4] * 4], [-2**63, -5, 0, 2**62], False),
    ("u32", 10, 2, [[2], [1, 1]], [0, 7, 70, 77, 99], True),
    ("u32", 256, 4, [[1, 3], [2, 2]], [0, 1, 256, 65536, 2**32 - 1], True),
    ("fixed_i64", 10, 3, [[3], [1, 2]], [100, 101, 210, 9, 990], True),
    ("i32", 256, 4, [[1, 3]], [-2**31, -1, 0, 1, 2**31 - 1], True),
]


def pin_signed_and_descending():
    """Beyond the paper: signed integers (offset binary) follow the integers'
    order, and descending order is the stable sort by decreasing key (equal
    keys in input order), against Python's stable sort on tiny inputs."""
    dts = {"u32": np.uint32, "fixed_i64": np.int64, "i32": np.int32, "i64": np.int64}
    for kind, base, ndims, groupings, alphabet, desc in _SIGNED_DESC_CASES:
        for alpha in itertools.combinations(alphabet, 3):
            for length in range(0, 4):
                for seq in itertools.product(alpha, repeat=length):
                    keys = np.array(seq, dtype=dts[kind])
                    vals = np.arange(length, dtype=np.uint32)
                    order = sorted(range(length), key=lambda i: int(seq[i]), reverse=desc)
                    for groups in groupings:
                        ko, vo, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups,
                                                descending=desc)
                        assert vo.tolist() == order, (kind, desc, groups, seq)
                        assert ko.tolist() == [int(seq[i]) for i in order]
                        ko2, _, _ = oracle.sort(keys, None, kind=kind, base=base, ndims=ndims, groups=groups,
                                                descending=desc)
                        assert ko2.tolist() == sorted((int(v) for v in seq), reverse=desc)
    # strings, descending: reverse memcmp order of the padded rows
    words = ["", "a", "ab", "b", "zz"]
    for alpha in itertools.combinations(words, 3):
        for length in range(0, 4):
            for seq in itertools.product(alpha, repeat=length):
                keys = _str_rows(seq, 2)
                rows = [bytes(r) for r in keys]
                order = sorted(range(length), key=lambda i: rows[i], reverse=True)
                vals = np.arange(length, dtype=np.uint32)
                for groups in ([2], [1, 1]):
                    ko, vo, _ = oracle.sort(keys, vals, kind="str", base=27, ndims=2, groups=groups,
                                            descending=True)
                    assert vo.tolist() == order, (seq, groups)


def pin_byte_strings():
    """Beyond the paper: 16-byte strings over every byte value (base 256, one
    dimension per byte) follow memcmp order, against Python's bytes order."""
    rng = np.random.default_rng(11)
    alphabet = [0, 1, ord("A"), ord("a"), 0x7F, 0x80, 0xFF]
    for trial in range(40):
        n = int(rng.integers(0, 40))
        keys = rng.choice(alphabet, size=(n, 4)).astype(np.uint8)
        keys[::3] = keys[0] if n else keys[::3]
        rows = [bytes(r) for r in keys]
        vals = np.arange(n, dtype=np.uint32)
        for desc in (False, True):
            order = sorted(range(n), key=lambda i: rows[i], reverse=desc)
            for groups in ([1, 1, 1, 1], [2, 2], [1, 3]):
                ko, vo, _ = oracle.sort(keys, vals, kind="str", base=256, ndims=4, groups=groups, descending=desc)
                assert vo.tolist() == order, (trial, desc, groups)
                assert [bytes(r) for r in ko] == [rows[i] for i in order]
                ko2, _, _ = oracle.sort(keys, None, kind="str", base=256, ndims=4, groups=groups, descending=desc)
                assert [bytes(r) for r in ko2] == sorted(rows, reverse=desc)


PINS = [pin_worked_example_output, pin_worked_example_hashing_state, pin_padding_example, pin_table3_shapes,
        pin_brute_force_tiny, pin_brute_force_strings, pin_medium_vs_library_stable_sort, pin_literal_walk_cost,
        pin_signed_and_descending, pin_byte_strings]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# Each mutation is (description, exact source text, replacement).
MUTANTS = [
    ("walk stops before the row maximum", "t <= sp->hmax[0] - sp->hmin[0]; t++", "t < sp->hmax[0] - sp->hmin[0]; t++"),
    ("inner walk bound exclusive", "if (!down && cur[j] < hi[j]) {", "if (!down && cur[j] + 1 < hi[j]) {"),
    ("H_Max comparison reversed", "if (sp->hmax[e] < coord[j]) sp->hmax[e] = coord[j];",
     "if (sp->hmax[e] > coord[j]) sp->hmax[e] = coord[j];"),
    ("H_Min never lowered", "} else if (sp->hmin[e] > coord[j]) {", "} else if (sp->hmin[e] < coord[j]) {"),
    ("digit index reversed", "return (uint32_t)((v / c->pw[n - 1 - j]) % c->d.base);\n  }\n  case ORC_U64",
     "return (uint32_t)((v / c->pw[j]) % c->d.base);\n  }\n  case ORC_U64"),
    ("rows walked descending", "const uint32_t r = down ? b - 1 - t : t;", "const uint32_t r = down ? t : b - 1 - t;"),
    ("descending inner coordinates restart at the minimum", "cur[j] = down ? hi[j] : lo[j];\n        j--;",
     "cur[j] = lo[j];\n        j--;"),
    ("descending one-dimensional walk ascends", "const uint64_t x = down ? sp->hmax[0] - t : sp->hmin[0] + t;",
     "const uint64_t x = sp->hmin[0] + t;"),
    ("signed 32-bit keys without the bias",
     "case ORC_I32: return (uint64_t)((int64_t)((const int32_t *)c->keys)[i] + 2147483648LL);",
     "case ORC_I32: return (uint64_t)(uint32_t)((const int32_t *)c->keys)[i];"),
    ("signed 64-bit keys without the bias",
     "case ORC_I64: return (uint64_t)((const int64_t *)c->keys)[i] ^ 0x8000000000000000ull;",
     "case ORC_I64: return (uint64_t)((const int64_t *)c->keys)[i];"),
    ("placement in reverse input order", "for (uint64_t i = 0; i < cnt; i++) {\n      uint64_t cell = element_cell",
     "for (uint64_t i = cnt; i-- > 0;) {\n      uint64_t cell = element_cell"),
    ("pad symbol sorts last", "return byte == 0 ? 0u : (uint32_t)(byte - 'a') + 1u;",
     "return byte == 0 ? 26u : (uint32_t)(byte - 'a');"),
    ("byte strings rebuilt from the 27-symbol alphabet", "  if (base == 256) return (uint8_t)sym;\n", ""),
    ("rebuilt key drops the prefix", "uint64_t v = prefix * c->pw[sp->w] + cell;", "uint64_t v = cell;"),
    ("untouched rows walked", "if (!sp->hmin_flag[row]) continue; /* row never touched */",
     "/* every row walked */"),
    ("single-element sub-arrays dropped", "if (s->vals_in == NULL) copy_key(s, base + st, items[st]);",
     "(void)0;"),
]


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutants_are_caught(mutant, tmp_path):
    desc, old, new = mutant
    src = oracle.source()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {desc}"
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path / "mutant.so"))
    caught = []
    with oracle.use_library(lib):
        for pin in PINS:
            try:
                pin()
            except (AssertionError, oracle.OracleError):
                caught.append(pin.__name__)
                break
    assert caught, f"no pin rejects the mutant '{desc}'"


def test_rejects_invalid_keys():
    with pytest.raises(oracle.OracleError):
        oracle.sort(np.array([10**6], np.uint32), None, kind="u32", base=10, ndims=6)
    with pytest.raises(oracle.OracleError):
        oracle.sort(np.array([-1], np.int64), None, kind="fixed_i64", base=10, ndims=3)
    with pytest.raises(oracle.OracleError):
        oracle.sort(_str_rows(["aB"], 2), None, kind="str", base=27, ndims=2)
    with pytest.raises(oracle.OracleError):  # groups must cover every dimension
        oracle.sort(np.array([1, 2], np.uint32), None, kind="u32", base=256, ndims=4, groups=[1, 2])


def test_empty_and_single():
    for n in (0, 1):
        keys = np.arange(n, dtype=np.uint32) + 5
        ko, vo, _ = oracle.sort(keys, np.arange(n, dtype=np.uint32), kind="u32", base=256, ndims=4,
                                groups=[1, 1, 1, 1])
        assert ko.tolist() == keys.tolist() and vo.tolist() == list(range(n))


def test_segments_match_per_array():
    keys, vals, offs = workloads.batched_u32(count=6, lo=1, hi=300)
    ko, vo, _ = oracle.sort_segments(keys, vals, offs, kind="u32", base=256, ndims=4, groups=[1, 1, 1, 1])
    for i in range(6):
        a, b = int(offs[i]), int(offs[i + 1])
        k1, v1, _ = oracle.sort(keys[a:b], vals[a:b], kind="u32", base=256, ndims=4, groups=[1, 1, 1, 1])
        assert np.array_equal(ko[a:b], k1) and np.array_equal(vo[a:b], v1)
