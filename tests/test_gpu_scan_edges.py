"""Sizes at the edges of the one-launch table scan of single arrays: the
count kernel's groups of 2, 4, 8 or 32 tiles with a short last group, and table
rows split into several 4096-tile segments with a short last segment.

At these sizes the output is checked by the properties that define a
stable sort with the input index as payload, on the device: keys
non-decreasing, equal keys in increasing index order, the values a
permutation of the indices, and every output key the input key its value
names."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api, workloads

pytestmark = pytest.mark.gpu

TILE = 8192  # keys per tile of the 512-thread prescanned passes (4-byte keys)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _library():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    B.rs_tuning_clear()


def _check_stable_sort(torch, keys_in, keys_out, vals_out, n):
    ki = keys_in[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    ko = keys_out[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    vo = vals_out[: 4 * n].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    assert bool((ko[1:] >= ko[:-1]).all()), "keys out of order"
    assert bool(((ko[1:] != ko[:-1]) | (vo[1:] > vo[:-1])).all()), "equal keys out of input order"
    assert bool((torch.sort(vo).values == torch.arange(n, device=vo.device)).all()), "values not a permutation"
    assert bool((ki[vo] == ko).all()), "a key moved without its value"


@pytest.mark.parametrize("n,base,ndims,what", [
    ((1 << 21) + 1, 256, 4, "one tile per count workgroup, one segment per row"),
    (1024 * TILE + 1, 256, 4, "2 tiles per count workgroup, last group of 1 tile"),
    (2048 * TILE + 1, 256, 4, "4 tiles per count workgroup, last group of 1 tile"),
    (8192 * TILE + 1, 256, 4, "8 tiles per count workgroup, last group of 1 tile, 3 segments"),
    (16388 * TILE - 5, 256, 4, "32 tiles per count workgroup, last group of 4 tiles, last segment of 4 tiles"),
    (9000 * TILE + 77, 10, 9, "100-cell passes (base 10), 8 tiles per count workgroup, short last group"),
])
def test_single_array_scan_edges(n, base, ndims, what):
    import torch
    _say(f"scan edges n={n} base={base}: {what}")
    d = B.key_desc("u32", base=base, ndims=ndims)
    assert B.rs_plan_inspect(d, n, True).form == B.RS_FORM_PRESCANNED
    w = workloads.uniform_u32_pairs(n, seed_extra=(n,))
    keys = w.keys % np.uint32(base ** ndims) if base ** ndims < (1 << 32) else w.keys
    kd, vd = api.to_device(keys), api.to_device(w.vals)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    tmp = api.empty_device(B.rs_temp_bytes(d, n, True))
    B.rs_sort_pairs(d, kd, ko, vd, vo, n, tmp, tmp.numel())
    torch.cuda.synchronize()
    _check_stable_sort(torch, kd, ko, vo, n)
