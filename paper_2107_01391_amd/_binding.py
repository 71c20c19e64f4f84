"""ctypes binding of librs.so: the C ABI of include/rs.h, names unchanged.

Argument marshalling only -- every step of the sort runs in the library's
HIP kernels.  Device pointers may be given as ints or as torch tensors
(their ``data_ptr()``); ``stream`` may be an int handle, a
``torch.cuda.Stream``, or None for torch's current stream.  A missing
library raises ``RSError``; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librs.so")

RS_OK = 0
RS_ERR_NULL_ARG = 1
RS_KEY_U32, RS_KEY_U64, RS_KEY_FIXED_I64, RS_KEY_STR, RS_KEY_I32, RS_KEY_I64 = 0, 1, 2, 3, 4, 5
RS_FLAG_VALIDATE = 1
RS_FLAG_DESCENDING = 2
RS_MAX_ELEMENTS = (1 << 30) - 1
RS_NOALLOC_SCRATCH_BYTES = 64 << 20

KINDS = {"u32": RS_KEY_U32, "u64": RS_KEY_U64, "fixed_i64": RS_KEY_FIXED_I64, "str": RS_KEY_STR,
         "i32": RS_KEY_I32, "i64": RS_KEY_I64}

EXPORTED = ["rs_temp_bytes", "rs_sort_keys", "rs_sort_pairs", "rs_sort_pairs_noalloc", "rs_batched_temp_bytes",
            "rs_sort_batched",
            "rs_status_string", "rs_last_error", "rs_prof_enable", "rs_prof_query",
            "rs_tuning_get", "rs_tuning_set", "rs_tuning_clear", "rs_tune_temp_bytes", "rs_tune_sort",
            "rs_tune_batched", "rs_tuning_save", "rs_tuning_load",
            "rs_graph_sort", "rs_graph_sort_batched", "rs_graph_launch", "rs_graph_destroy",
            "rs_server_work_bytes", "rs_server_create", "rs_server_submit", "rs_server_poll", "rs_server_wait",
            "rs_server_result", "rs_server_release", "rs_server_get_stats", "rs_server_reset_stats",
            "rs_server_clock", "rs_server_destroy", "rs_server_collect", "rs_plan_inspect"]
RS_ERR_BUSY = 8
RS_SERVE_BATCHED, RS_SERVE_PER_REQUEST = 0, 1


class RSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class KeyDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("base", ctypes.c_uint32), ("ndims", ctypes.c_uint32),
                ("frac_digits", ctypes.c_uint32), ("str_width", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


def key_desc(kind: str | int, base: int = 0, ndims: int = 0, frac_digits: int = 0, str_width: int = 0,
             validate: bool = False, descending: bool = False) -> KeyDesc:
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    if k == RS_KEY_STR and not str_width:
        str_width = 16
    flags = (RS_FLAG_VALIDATE if validate else 0) | (RS_FLAG_DESCENDING if descending else 0)
    return KeyDesc(k, base, ndims, frac_digits, str_width, flags)


class Tuning(ctypes.Structure):
    """rs_tuning: how the digits are grouped into passes and the tile shape."""
    _fields_ = [("digit_bits", ctypes.c_uint32), ("max_cells", ctypes.c_uint32), ("tile_block", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("prescan_min_n", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


RS_FORM_LOCAL, RS_FORM_LITERAL, RS_FORM_CHAINED, RS_FORM_PRESCANNED = 0, 1, 2, 3


class PlanInfo(ctypes.Structure):
    """rs_plan_info: the form a sort takes and, for the literal form, where
    its counts, traverse maps and starts lie in tmp."""
    _fields_ = [("form", ctypes.c_uint32), ("passes", ctypes.c_uint32), ("tile_keys", ctypes.c_uint32),
                ("literal_cells", ctypes.c_uint32), ("map_rows", ctypes.c_uint32), ("map_inner", ctypes.c_uint32),
                ("scan_chunk", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("off_counts", ctypes.c_uint64),
                ("off_map_lo", ctypes.c_uint64), ("off_map_hi", ctypes.c_uint64), ("off_starts", ctypes.c_uint64),
                ("tmp_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ServerConfig(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint64), ("max_slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("with_values", ctypes.c_uint32),
                ("min_batch", ctypes.c_uint32), ("batch_max_n", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("keys_sorted", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("busy", ctypes.c_uint64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("span_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str | None = None):
    """Loads librs.so (once).  Raises RSError when it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RSError(-1, f"{p} is missing: build it with `python -m paper_2107_01391_amd.build_lib` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(p)
    vp, u64, u32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
    dp = ctypes.POINTER(KeyDesc)
    lib.rs_temp_bytes.argtypes = [dp, u64, ctypes.c_int, ctypes.POINTER(sz)]
    lib.rs_sort_keys.argtypes = [dp, vp, vp, u64, vp, sz, vp]
    lib.rs_sort_pairs.argtypes = [dp, vp, vp, vp, vp, u64, vp, sz, vp]
    lib.rs_sort_pairs_noalloc.argtypes = [dp, vp, vp, vp, vp, u64, vp]
    lib.rs_batched_temp_bytes.argtypes = [dp, u64, u32, ctypes.c_int, ctypes.POINTER(sz)]
    lib.rs_sort_batched.argtypes = [dp, vp, vp, vp, vp, vp, u32, u64, vp, sz, vp]
    for f in ("rs_temp_bytes", "rs_sort_keys", "rs_sort_pairs", "rs_sort_pairs_noalloc", "rs_batched_temp_bytes",
              "rs_sort_batched"):
        getattr(lib, f).restype = ctypes.c_int
    lib.rs_status_string.argtypes = [ctypes.c_int]
    lib.rs_status_string.restype = ctypes.c_char_p
    lib.rs_last_error.argtypes = []
    lib.rs_last_error.restype = ctypes.c_char_p
    lib.rs_prof_enable.argtypes = [ctypes.c_int]
    lib.rs_prof_enable.restype = ctypes.c_int
    lib.rs_prof_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)]
    lib.rs_prof_query.restype = ctypes.c_int
    tp = ctypes.POINTER(Tuning)
    dbl = ctypes.POINTER(ctypes.c_double)
    ci = ctypes.c_int
    lib.rs_tuning_get.argtypes = [dp, u64, ci, ci, tp]
    lib.rs_tuning_set.argtypes = [dp, u64, ci, ci, tp]
    lib.rs_tuning_clear.argtypes = []
    lib.rs_tune_temp_bytes.argtypes = [dp, u64, u32, ci, ctypes.POINTER(sz)]
    lib.rs_tune_sort.argtypes = [dp, vp, vp, vp, vp, u64, vp, sz, vp, u32, tp, dbl]
    lib.rs_tune_batched.argtypes = [dp, vp, vp, vp, vp, vp, u32, u64, vp, sz, vp, u32, tp, dbl]
    lib.rs_tuning_save.argtypes = [ctypes.c_char_p]
    lib.rs_tuning_load.argtypes = [ctypes.c_char_p]
    gp = ctypes.POINTER(vp)
    lib.rs_graph_sort.argtypes = [dp, vp, vp, vp, vp, u64, vp, sz, gp]
    lib.rs_graph_sort_batched.argtypes = [dp, vp, vp, vp, vp, vp, u32, u64, vp, sz, gp]
    lib.rs_graph_launch.argtypes = [vp, vp]
    lib.rs_graph_destroy.argtypes = [vp]
    for f in ("rs_tuning_get", "rs_tuning_set", "rs_tuning_clear", "rs_tune_temp_bytes", "rs_tune_sort",
              "rs_tune_batched", "rs_tuning_save", "rs_tuning_load", "rs_graph_sort", "rs_graph_sort_batched",
              "rs_graph_launch", "rs_graph_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    cp = ctypes.POINTER(ServerConfig)
    u64p = ctypes.POINTER(u64)
    lib.rs_server_work_bytes.argtypes = [dp, cp, ctypes.POINTER(sz)]
    lib.rs_server_create.argtypes = [dp, cp, vp, vp, vp, vp, vp, sz, gp]
    lib.rs_server_submit.argtypes = [vp, vp, vp, u64, u64, vp, u64p]
    lib.rs_server_poll.argtypes = [vp, u64, ctypes.POINTER(ci)]
    lib.rs_server_wait.argtypes = [vp, u64]
    lib.rs_server_result.argtypes = [vp, u64, u64p, u64p]
    lib.rs_server_release.argtypes = [vp, u64]
    lib.rs_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.rs_server_reset_stats.argtypes = [vp]
    lib.rs_server_clock.argtypes = [u64p]
    lib.rs_server_destroy.argtypes = [vp]
    lib.rs_server_collect.argtypes = [vp, u64p, u32, ctypes.POINTER(u32), u32]
    for f in ("rs_server_work_bytes", "rs_server_create", "rs_server_submit", "rs_server_poll", "rs_server_wait",
              "rs_server_result", "rs_server_release", "rs_server_get_stats", "rs_server_reset_stats",
              "rs_server_clock", "rs_server_destroy", "rs_server_collect"):
        getattr(lib, f).restype = ctypes.c_int
    lib.rs_plan_inspect.argtypes = [dp, u64, ci, ctypes.POINTER(PlanInfo)]
    lib.rs_plan_inspect.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s) -> int | None:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(st: int):
    if st != RS_OK:
        lib = load_library()
        raise RSError(st, f"{lib.rs_status_string(st).decode()}: {lib.rs_last_error().decode()}")


def rs_status_string(status: int) -> str:
    return load_library().rs_status_string(status).decode()


def rs_last_error() -> str:
    return load_library().rs_last_error().decode()


def rs_temp_bytes(desc: KeyDesc, n: int, with_values: bool) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().rs_temp_bytes(ctypes.byref(desc), n, int(bool(with_values)), ctypes.byref(out)))
    return out.value


def rs_sort_keys(desc: KeyDesc, keys_in, keys_out, n: int, tmp, tmp_bytes: int, stream=None) -> None:
    _check(load_library().rs_sort_keys(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), n, _ptr(tmp), tmp_bytes,
                                       _stream(stream)))


def rs_sort_pairs(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, n: int, tmp, tmp_bytes: int,
                  stream=None) -> None:
    _check(load_library().rs_sort_pairs(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                        _ptr(vals_out), n, _ptr(tmp), tmp_bytes, _stream(stream)))


def rs_sort_pairs_noalloc(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, n: int, stream=None) -> None:
    """rs_sort_pairs with the library's static device scratch (no tmp)."""
    _check(load_library().rs_sort_pairs_noalloc(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                                _ptr(vals_out), n, _stream(stream)))


def rs_plan_inspect(desc: KeyDesc, n: int, with_values: bool) -> PlanInfo:
    info = PlanInfo()
    _check(load_library().rs_plan_inspect(ctypes.byref(desc), n, int(bool(with_values)), ctypes.byref(info)))
    return info


def rs_batched_temp_bytes(desc: KeyDesc, total: int, nseg: int, with_values: bool) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().rs_batched_temp_bytes(ctypes.byref(desc), total, nseg, int(bool(with_values)),
                                                ctypes.byref(out)))
    return out.value


def rs_sort_batched(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, nseg: int, total: int, tmp,
                    tmp_bytes: int, stream=None) -> None:
    _check(load_library().rs_sort_batched(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                          _ptr(vals_out), _ptr(d_seg_offsets), nseg, total, _ptr(tmp), tmp_bytes,
                                          _stream(stream)))


def rs_prof_enable(enable: bool) -> None:
    """Starts (discarding earlier records) or stops per-kernel event timing."""
    _check(load_library().rs_prof_enable(int(bool(enable))))


def rs_prof_query(name: str) -> tuple[int, float]:
    """(launches, total milliseconds) of kernel `name` since timing started."""
    n = ctypes.c_uint64(0)
    ms = ctypes.c_double(0.0)
    _check(load_library().rs_prof_query(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ------------------------------------------------------------------ tuning

def rs_tuning_get(desc: KeyDesc, n: int, with_values: bool, batched: bool = False) -> Tuning:
    t = Tuning()
    _check(load_library().rs_tuning_get(ctypes.byref(desc), n, int(bool(with_values)), int(bool(batched)),
                                        ctypes.byref(t)))
    return t


def rs_tuning_set(desc: KeyDesc, n: int, with_values: bool, batched: bool, t: Tuning) -> None:
    _check(load_library().rs_tuning_set(ctypes.byref(desc), n, int(bool(with_values)), int(bool(batched)),
                                        ctypes.byref(t)))


def rs_tuning_clear() -> None:
    _check(load_library().rs_tuning_clear())


def rs_tune_temp_bytes(desc: KeyDesc, n: int, nseg: int, with_values: bool) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().rs_tune_temp_bytes(ctypes.byref(desc), n, nseg, int(bool(with_values)), ctypes.byref(out)))
    return out.value


def rs_tune_sort(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, n: int, tmp, tmp_bytes: int, stream=None,
                 reps: int = 3) -> tuple[Tuning, float]:
    t, ms = Tuning(), ctypes.c_double(0.0)
    _check(load_library().rs_tune_sort(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                       _ptr(vals_out), n, _ptr(tmp), tmp_bytes, _stream(stream), reps,
                                       ctypes.byref(t), ctypes.byref(ms)))
    return t, ms.value


def rs_tune_batched(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, nseg: int, total: int, tmp,
                    tmp_bytes: int, stream=None, reps: int = 3) -> tuple[Tuning, float]:
    t, ms = Tuning(), ctypes.c_double(0.0)
    _check(load_library().rs_tune_batched(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                          _ptr(vals_out), _ptr(d_seg_offsets), nseg, total, _ptr(tmp), tmp_bytes,
                                          _stream(stream), reps, ctypes.byref(t), ctypes.byref(ms)))
    return t, ms.value


def rs_tuning_save(path: str) -> None:
    _check(load_library().rs_tuning_save(path.encode()))


def rs_tuning_load(path: str) -> None:
    _check(load_library().rs_tuning_load(path.encode()))


# ------------------------------------------------------------------ graphs

class Graph:
    """A captured sort (rs_graph); replay with launch(), free with close()."""

    def __init__(self, handle: int, keep: tuple):
        self._h = handle
        self._keep = keep  # the buffers the graph points at stay alive with it

    def launch(self, stream=None) -> None:
        if not self._h:
            raise RSError(RS_ERR_NULL_ARG, "graph is closed")
        _check(load_library().rs_graph_launch(self._h, _stream(stream)))

    def close(self) -> None:
        if self._h:
            _check(load_library().rs_graph_destroy(self._h))
            self._h = None
            self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rs_graph_sort(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, n: int, tmp, tmp_bytes: int) -> Graph:
    h = ctypes.c_void_p(None)
    _check(load_library().rs_graph_sort(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                        _ptr(vals_out), n, _ptr(tmp), tmp_bytes, ctypes.byref(h)))
    return Graph(h.value, (keys_in, keys_out, vals_in, vals_out, tmp))


def rs_graph_sort_batched(desc: KeyDesc, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, nseg: int, total: int,
                          tmp, tmp_bytes: int) -> Graph:
    h = ctypes.c_void_p(None)
    _check(load_library().rs_graph_sort_batched(ctypes.byref(desc), _ptr(keys_in), _ptr(keys_out), _ptr(vals_in),
                                                _ptr(vals_out), _ptr(d_seg_offsets), nseg, total, _ptr(tmp),
                                                tmp_bytes, ctypes.byref(h)))
    return Graph(h.value, (keys_in, keys_out, vals_in, vals_out, d_seg_offsets, tmp))
