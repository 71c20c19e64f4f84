"""CPU oracle of Recombinant Sort -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper over ``rs_oracle.c``: a plain single-threaded C
implementation of the paper's hashing cycle (Section 3.1, eq. (1)),
extraction walk (Section 3.2) and stable placement, applied level by level
over groups of digit dimensions.  Only ``tests/``, the package smoke check and
the benchmark's CPU-baseline leg may import this module; the GPU library never
does, and the two share no code.

Default dimension groups per workload (most significant group first):

=====================  ===========  =======================================
workload               groups       meaning
=====================  ===========  =======================================
uniform_decimal_u32    [6]          one literal 10**6-cell space
uniform_u32_pairs      [1, 3]       256 buckets, then a 2**24-cell space each
fixed_point_decimals   [3, 6]       10**3 buckets, then 10**6 cells each
strings16              [2] * 8      27**2 = 729 cells per level
batched_u32            [1, 1, 1, 1] per array, 256 cells per level
=====================  ===========  =======================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND = {"u32": 0, "u64": 1, "fixed_i64": 2, "str": 3, "i32": 4, "i64": 5}
ERRORS = {1: "bad argument", 2: "key outside the count space", 3: "count space too large",
          4: "out of memory", 5: "loop invariant violated"}

DEFAULT_GROUPS = {
    "uniform_decimal_u32": [6],
    "uniform_u32_pairs": [1, 3],
    "fixed_point_decimals": [3, 6],
    "strings16": [2] * 8,
    "batched_u32": [1, 1, 1, 1],
}


class OracleError(RuntimeError):
    pass


class _Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("base", ctypes.c_uint32),
                ("ndims", ctypes.c_uint32), ("str_width", ctypes.c_uint32), ("order", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("cells_visited", ctypes.c_uint64), ("spaces", ctypes.c_uint64),
                ("max_depth", ctypes.c_uint64)]


@dataclass
class Stats:
    cells_visited: int  # k, summed over every extraction walk
    spaces: int         # hashing cycles run
    max_depth: int      # hierarchy levels used


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc -O2 into ``oracle/liboracle.so``."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC],
                   check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.orc_sort.argtypes = [ctypes.POINTER(_Desc), vp, vp, vp, vp, u64, vp, u32, ctypes.POINTER(_Stats)]
    lib.orc_sort.restype = ctypes.c_int
    lib.orc_sort_segments.argtypes = [ctypes.POINTER(_Desc), vp, vp, vp, vp, vp, u32, vp, u32,
                                      ctypes.POINTER(_Stats)]
    lib.orc_sort_segments.restype = ctypes.c_int
    lib.orc_hash_level.argtypes = [ctypes.POINTER(_Desc), vp, u64, u32, u32, vp, vp, vp, vp, vp, vp]
    lib.orc_hash_level.restype = ctypes.c_int
    lib.orc_dims_for.argtypes = [u64, u32]
    lib.orc_dims_for.restype = u32
    return lib


_lib = None
_override = None


def _load():
    global _lib
    if _override is not None:
        return _override
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(_LIB)
    return _lib


class use_library:
    """Context manager: route this module's calls to another build of the
    oracle (the tests use it to show that the pins reject mutated builds)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _override
        self._prev = _override
        _override = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _override
        _override = self._prev
        return False


def build_variant(source_text: str, out_path: str) -> str:
    """Compiles an edited copy of the oracle source (tests only)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-w", "-shared", "-fPIC", "-o", out_path, src], check=True)
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def _desc(kind: str, base: int, ndims: int, str_width: int = 0, descending: bool = False) -> _Desc:
    return _Desc(KIND[kind], base, ndims, str_width, 1 if descending else 0)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int):
    if rc != 0:
        raise OracleError(f"oracle error {rc}: {ERRORS.get(rc, '?')}")


def _key_array(keys: np.ndarray, kind: str) -> np.ndarray:
    want = {"u32": np.uint32, "u64": np.uint64, "fixed_i64": np.int64, "str": np.uint8, "i32": np.int32,
            "i64": np.int64}[kind]
    return np.ascontiguousarray(keys, dtype=want)


def sort(keys: np.ndarray, vals: np.ndarray | None = None, *, kind: str, base: int, ndims: int,
         groups: list[int] | None = None, str_width: int = 0, descending: bool = False):
    """Returns (keys_out, vals_out or None, Stats).  Stable, ascending (or
    descending: the mirrored walk, equal keys still in input order)."""
    lib = _load()
    keys = _key_array(keys, kind)
    n = keys.shape[0]
    if kind == "str":
        str_width = keys.shape[1] if keys.ndim == 2 else str_width
    groups = [ndims] if groups is None else list(groups)
    g = np.asarray(groups, dtype=np.uint32)
    out = np.empty_like(keys)
    vin = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32)
    vout = None if vin is None else np.empty_like(vin)
    st = _Stats()
    d = _desc(kind, base, ndims, str_width, descending)
    _check(lib.orc_sort(ctypes.byref(d), _ptr(keys), _ptr(out), _ptr(vin), _ptr(vout), n, _ptr(g), len(groups),
                        ctypes.byref(st)))
    return out, vout, Stats(st.cells_visited, st.spaces, st.max_depth)


def sort_segments(keys: np.ndarray, vals: np.ndarray | None, offsets: np.ndarray, *, kind: str, base: int,
                  ndims: int, groups: list[int] | None = None, str_width: int = 0, descending: bool = False):
    """Sorts each segment [offsets[i], offsets[i+1]) on its own."""
    lib = _load()
    keys = _key_array(keys, kind)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    groups = [ndims] if groups is None else list(groups)
    g = np.asarray(groups, dtype=np.uint32)
    out = np.empty_like(keys)
    vin = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32)
    vout = None if vin is None else np.empty_like(vin)
    st = _Stats()
    d = _desc(kind, base, ndims, str_width or (keys.shape[1] if keys.ndim == 2 else 0), descending)
    _check(lib.orc_sort_segments(ctypes.byref(d), _ptr(keys), _ptr(out), _ptr(vin), _ptr(vout), _ptr(offs),
                                 len(offs) - 1, _ptr(g), len(groups), ctypes.byref(st)))
    return out, vout, Stats(st.cells_visited, st.spaces, st.max_depth)


def hash_level(keys: np.ndarray, *, kind: str, base: int, ndims: int, dlo: int = 0, w: int | None = None,
               str_width: int = 0) -> dict:
    """One hashing cycle + extraction walk over the whole input.

    Returns S (shape [base]*w), start (same shape, 0 for empty cells), the
    traverse maps (``hmin_flag``/``hmin``/``hmax``: one entry for w == 1,
    shape [base, w-1] otherwise) and k, the number of cells walked."""
    lib = _load()
    keys = _key_array(keys, kind)
    w = ndims - dlo if w is None else w
    cells = base**w
    entries = 1 if w == 1 else base * (w - 1)
    S = np.zeros(cells, np.uint64)
    start = np.zeros(cells, np.uint64)
    hf = np.zeros(entries, np.uint32)
    hmin = np.zeros(entries, np.uint32)
    hmax = np.zeros(entries, np.uint32)
    k = np.zeros(1, np.uint64)
    d = _desc(kind, base, ndims, str_width or (keys.shape[1] if keys.ndim == 2 else 0))
    _check(lib.orc_hash_level(ctypes.byref(d), _ptr(keys), keys.shape[0], dlo, w, _ptr(S), _ptr(start), _ptr(hf),
                              _ptr(hmin), _ptr(hmax), _ptr(k)))
    shape = (base,) * w
    mshape = (1,) if w == 1 else (base, w - 1)
    return {"S": S.reshape(shape), "start": start.reshape(shape), "hmin_flag": hf.reshape(mshape),
            "hmin": hmin.reshape(mshape), "hmax": hmax.reshape(mshape), "k": int(k[0])}


def dims_for(max_exclusive: int, base: int = 10) -> int:
    """Digits per key for values below ``max_exclusive`` (Table 3)."""
    return int(_load().orc_dims_for(max_exclusive, base))


def timed_sort(*args, **kwargs):
    """sort() plus its wall-clock seconds (single thread)."""
    t0 = time.perf_counter()
    r = sort(*args, **kwargs)
    return r, time.perf_counter() - t0
