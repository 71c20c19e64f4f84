"""Shared helpers of the GPU tests: run the HIP library through its C ABI on
seeded workloads and run the CPU oracle on the same host buffers."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2107_01391_amd import _binding as B
from paper_2107_01391_amd import api

KEY_DTYPE = {"u32": np.uint32, "u64": np.uint64, "fixed_i64": np.int64, "i32": np.int32, "i64": np.int64}


def desc_of(kind, base, ndims, str_width=0, frac_digits=0, validate=False, descending=False):
    return B.key_desc(kind, base=base, ndims=ndims, frac_digits=frac_digits, str_width=str_width,
                      validate=validate, descending=descending)


def key_shape(kind, n):
    return (n, 16) if kind == "str" else (n,)


def key_dtype(kind):
    return np.uint8 if kind == "str" else KEY_DTYPE[kind]


def gpu_sort(keys: np.ndarray, vals: np.ndarray | None, kind: str, base: int, ndims: int, *, in_place=False,
             validate=False, frac_digits=0, descending=False):
    """Sorts on cuda:0 through rs_sort_pairs / rs_sort_keys; returns host arrays."""
    import torch
    n = keys.shape[0]
    d = desc_of(kind, base, ndims, 16 if kind == "str" else 0, frac_digits, validate, descending)
    kd = api.to_device(keys)
    ko = kd if in_place else api.empty_device(kd.numel())
    if vals is None:
        need = B.rs_temp_bytes(d, n, False)
        tmp = api.empty_device(need)
        B.rs_sort_keys(d, kd, ko, n, tmp, tmp.numel())
        torch.cuda.synchronize()
        return api.to_host(ko, key_dtype(kind), key_shape(kind, n)), None
    vd = api.to_device(vals)
    vo = vd if in_place else api.empty_device(vd.numel())
    need = B.rs_temp_bytes(d, n, True)
    tmp = api.empty_device(need)
    B.rs_sort_pairs(d, kd, ko, vd, vo, n, tmp, tmp.numel())
    torch.cuda.synchronize()
    return api.to_host(ko, key_dtype(kind), key_shape(kind, n)), api.to_host(vo, np.uint32, (n,))


def oracle_sort(keys, vals, kind, base, ndims, groups=None, descending=False):
    if groups is None:
        groups = fast_groups(kind, base, ndims)
    ko, vo, _ = oracle.sort(keys, vals, kind=kind, base=base, ndims=ndims, groups=groups, descending=descending)
    return ko, vo


def fast_groups(kind, base, ndims):
    """Dimension groups that keep the oracle quick at test sizes (its output
    does not depend on the grouping; the oracle pins check that)."""
    if kind == "str":
        return [2] * 8 if base == 27 else [1] * 16
    cells, w = 1, 0
    while w < ndims and cells * base <= 1024:
        cells *= base
        w += 1
    w = max(w, 1)
    groups = []
    left = ndims
    while left > 0:
        groups.append(min(w, left))
        left -= groups[-1]
    return groups


def assert_same(gk, gv, ok, ov, what=""):
    assert gk.shape == ok.shape, what
    if not np.array_equal(gk, ok):
        bad = np.nonzero((gk != ok).reshape(gk.shape[0], -1).any(axis=1))[0]
        raise AssertionError(f"{what}: keys differ at {bad.size} positions, first {bad[:8].tolist()}")
    if ov is not None:
        if not np.array_equal(gv, ov):
            bad = np.nonzero(gv != ov)[0]
            raise AssertionError(f"{what}: values differ at {bad.size} positions, first {bad[:8].tolist()}")
