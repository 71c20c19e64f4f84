"""Per-kernel pins of the literal form (keys only on a small space).

The kernels' intermediate state is read back from the scratch buffer after
the sort, at the offsets rs_plan_inspect reports, and compared element by
element with the oracle's hashing cycle and walk:

- the count of every cell against the oracle's S (eq. (1));
- the traverse maps (Section 3.1) against the oracle's H_Min / H_Max: for a
  two-dimensional space the GPU's per-row occupied range is exactly the
  oracle's (touched flag, least and greatest column); for more dimensions
  it is each row's occupied range of cell offsets, taken from S;
- the starts (Section 3.2's running position) of occupied cells against the
  oracle's;
- the walk's trimming: the scratch is poisoned before the sort, and the
  starts of every 4096-cell chunk that no row's occupied range reaches must
  still hold the poison (the chunk was neither read nor written), while
  every other chunk's starts were written.
"""
from __future__ import annotations

import json
import os
import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
POISON = 0xA5A5A5A5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    B.rs_tuning_clear()


def _keys(case):
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    if case == "worked_example":
        # the worked example's ten keys (one fractional digit, scaled by 10),
        # repeated so that the literal form (more than 4096 keys) is chosen
        with open(os.path.join(HERE, "golden", "worked_example.json")) as f:
            ex = json.load(f)["worked_example"]
        one = np.array([int(round(float(x) * 10)) for x in ex["input"]], np.uint32)
        return np.tile(one, 500), 10, 2, ex
    if case == "two_dim_rows":
        # 37 of 1000 rows, each with its own column range
        rows = rng.choice(1000, 37, replace=False)
        lo = rng.integers(0, 900, 37)
        width = rng.integers(1, 100, 37)
        pick = rng.integers(0, 37, 300_000)
        cols = lo[pick] + (rng.random(300_000) * width[pick]).astype(np.int64)
        return (rows[pick] * 1000 + cols).astype(np.uint32), 1000, 2, None
    if case == "clustered_six_dim":
        # 2^22 keys inside 1/256 of a 2^24-cell space (hex digits)
        return rng.integers(0x350000, 0x360000, 1 << 22, dtype=np.uint32), 16, 6, None
    if case == "three_dim_sparse":
        rows = np.array([3, 41, 97])
        pick = rng.integers(0, 3, 400_000)
        inner = rng.integers(100, 2000, 400_000)
        return (rows[pick] * 10_000 + inner).astype(np.uint32), 100, 3, None
    raise ValueError(case)


@pytest.mark.parametrize("case", ["worked_example", "two_dim_rows", "clustered_six_dim", "three_dim_sparse"])
def test_literal_counts_maps_starts_and_skipped_chunks(case):
    import torch
    keys, base, ndims, ex = _keys(case)
    n = keys.shape[0]
    _say(f"literal maps {case}: n={n} base={base} ndims={ndims}")
    d = B.key_desc("u32", base=base, ndims=ndims)
    info = B.rs_plan_inspect(d, n, False)
    assert info.form == B.RS_FORM_LITERAL
    cells, rows, inner, chunk = info.literal_cells, info.map_rows, info.map_inner, info.scan_chunk
    assert cells == base ** ndims and rows == base
    words = (info.tmp_bytes + 3) // 4
    tmp = torch.full((words,), POISON - (1 << 32), dtype=torch.int32, device="cuda")  # the poison, as int32
    kd = api.to_device(keys)
    ko = torch.empty_like(kd)
    B.rs_sort_keys(d, kd, ko, n, tmp, info.tmp_bytes)
    torch.cuda.synchronize()
    out = api.to_host(ko, np.uint32, (n,))
    t = tmp.cpu().numpy().view(np.uint32)
    counts = t[info.off_counts // 4: info.off_counts // 4 + cells]
    nlo = t[info.off_map_lo // 4: info.off_map_lo // 4 + rows]
    hi = t[info.off_map_hi // 4: info.off_map_hi // 4 + rows]
    starts = t[info.off_starts // 4: info.off_starts // 4 + cells]

    assert np.array_equal(out, np.sort(keys))
    ref = oracle.hash_level(keys, kind="u32", base=base, ndims=ndims)
    S = ref["S"].reshape(-1)
    # the hashing cycle: every cell's count
    assert np.array_equal(counts.astype(np.uint64), S)

    # the traverse maps
    touched = nlo != 0
    lo = ~nlo
    occ = S.reshape(rows, inner) > 0
    assert np.array_equal(touched, occ.any(axis=1))
    for r in np.nonzero(touched)[0]:
        offs = np.nonzero(occ[r])[0]
        assert lo[r] == offs[0] and hi[r] == offs[-1], f"row {r}"
    assert np.all(hi[~touched] == 0)
    if ndims == 2:
        # exactly the oracle's H_Min (flag, least column) and H_Max
        hf, hmin, hmax = ref["hmin_flag"][:, 0], ref["hmin"][:, 0], ref["hmax"][:, 0]
        assert np.array_equal(touched, hf == 1)
        assert np.array_equal(lo[touched], hmin[touched])
        assert np.array_equal(hi[touched], hmax[touched])
    if ex is not None:
        # and the values the paper prints for its example
        assert hi.tolist() == ex["H_Max"]
        assert [[int(touched[r]), int(lo[r]) if touched[r] else 0] for r in range(rows)] == ex["H_Min"]

    # the walk: starts of occupied cells, and the chunks it skipped
    occupied_cells = S > 0
    assert np.array_equal(starts[occupied_cells].astype(np.uint64), ref["start"].reshape(-1)[occupied_cells])
    nchunks = (cells + chunk - 1) // chunk
    reached = np.zeros(nchunks, bool)
    for r in np.nonzero(touched)[0]:
        first, last = r * inner + int(lo[r]), r * inner + int(hi[r])
        reached[first // chunk: last // chunk + 1] = True
    skipped = 0
    for c in range(nchunks):
        seg = starts[c * chunk: min(cells, (c + 1) * chunk)]
        if reached[c]:
            assert not np.all(seg == POISON), f"chunk {c} reached but not written"
        else:
            assert np.all(seg == POISON), f"chunk {c} skipped but written"
            skipped += 1
    _say(f"  {skipped} of {nchunks} chunks skipped")
    if case in ("two_dim_rows", "clustered_six_dim", "three_dim_sparse"):
        assert skipped > 0
