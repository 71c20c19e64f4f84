"""CPU-only checks of the C-ABI library: it loads without a GPU, exports every
symbol include/rs.h declares, and its host-side planning and argument
validation behave as documented.  No kernel is launched."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_2107_01391_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        names |= set(re.findall(r"^\s*(?:rs_status|const char \*)\s*(rs_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_header_declares_the_binding_names():
    assert _declared() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r" T (rs_\w+)", out.stdout))
    assert set(_declared()) <= exported


def test_status_strings():
    for st in range(0, 9):
        assert B.rs_status_string(st)
    assert B.rs_status_string(12345) == "unknown status"


@pytest.mark.parametrize("kind,base,ndims,n,pairs", [
    ("u32", 256, 4, 1 << 28, True), ("u32", 10, 6, 10**6, False), ("fixed_i64", 10, 9, 10**8, True),
    ("str", 27, 16, 1 << 24, True), ("u64", 256, 8, 1000, True), ("u32", 0, 0, 5, False), ("u32", 16, 8, 77, True),
])
def test_temp_bytes_plans(kind, base, ndims, n, pairs):
    d = B.key_desc(kind, base=base, ndims=ndims)
    t = B.rs_temp_bytes(d, n, pairs)
    key_bytes = {"u32": 4, "u64": 8, "fixed_i64": 8, "str": 16}[kind]
    assert t % 256 == 0
    # scratch is O(n): one alternate copy of the keys (and values), the
    # look-back words, and small tables
    assert t < n * (key_bytes + 4) * 2 + (64 << 20)


def test_zero_length_needs_no_pointers():
    d = B.key_desc("u32")
    lib = B.load_library()
    assert lib.rs_sort_pairs(ctypes.byref(d), None, None, None, None, 0, None, 0, None) == 0
    assert lib.rs_sort_keys(ctypes.byref(d), None, None, 0, None, 0, None) == 0


@pytest.mark.parametrize("desc,n,status", [
    (dict(kind="str", str_width=8), 10, 5),              # only 16-byte strings
    (dict(kind="str", base=10), 10, 2),                  # strings are base 27
    (dict(kind="u32", base=10, ndims=11), 10, 2),        # 10 digits already fill u32
    (dict(kind="u32", base=1), 10, 2),
    (dict(kind=7), 10, 2),
    (dict(kind="u32"), 1 << 30, 5),                      # above RS_MAX_ELEMENTS
])
def test_bad_descriptions(desc, n, status):
    kind = desc.pop("kind")
    d = B.key_desc(kind, **desc)
    with pytest.raises(B.RSError) as e:
        B.rs_temp_bytes(d, n, True)
    assert e.value.status == status
    assert B.rs_last_error()


def test_null_and_small_tmp_rejected_before_launch():
    d = B.key_desc("u32")
    lib = B.load_library()
    assert lib.rs_sort_pairs(ctypes.byref(d), None, None, None, None, 10, None, 0, None) == 1
    fake = ctypes.c_void_p(256)  # never dereferenced: the size check fails first
    need = B.rs_temp_bytes(d, 1000, True)
    st = lib.rs_sort_pairs(ctypes.byref(d), fake, fake, fake, fake, 1000, fake, need - 256, None)
    assert st == 4
    assert lib.rs_sort_pairs(None, fake, fake, fake, fake, 1000, fake, need, None) == 1


@pytest.mark.parametrize("kind,kptr,vptr,tptr", [
    ("u32", 258, 512, 1024),   # keys off their 4-byte size
    ("u64", 260, 512, 1024),   # keys off their 8-byte size
    ("str", 264, 512, 1024),   # 16-byte rows off 16 bytes
    ("u32", 256, 514, 1024),   # values off 4 bytes
    ("u32", 256, 512, 1028),   # tmp off 256 bytes
])
def test_misaligned_pointers_rejected_before_launch(kind, kptr, vptr, tptr):
    """Pointers are never dereferenced: the alignment check fails first."""
    d = B.key_desc(kind)
    lib = B.load_library()
    need = B.rs_temp_bytes(d, 1000, True)
    k, v, t = (ctypes.c_void_p(x) for x in (kptr, vptr, tptr))
    assert lib.rs_sort_pairs(ctypes.byref(d), k, k, v, v, 1000, t, need, None) == 5
    assert "align" in B.rs_last_error()
    offs = ctypes.c_void_p(2048)
    need_b = B.rs_batched_temp_bytes(d, 1000, 4, True)
    assert lib.rs_sort_batched(ctypes.byref(d), k, k, v, v, offs, 4, 1000, t, need_b, None) == 5


def test_codec_host_build(tmp_path):
    """The digit codecs, built for the host from the same header the kernels
    use, against plain division / byte arithmetic on edge and random values."""
    src = os.path.join(ROOT, "tests", "codec_check.cpp")
    exe = str(tmp_path / "codec_check")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", "-I",
                    os.path.join(ROOT, "paper_2107_01391_amd", "csrc"), src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "codec ok" in r.stdout


def test_seg_bounds_host_build(tmp_path):
    """The batched form's resolution of the caller's offsets (the arithmetic
    of rs_seg_plan), built for the host from the header the kernel uses:
    valid offsets pass unchanged; any offsets stay inside the buffers and the
    scratch's tile bound."""
    src = os.path.join(ROOT, "tests", "seg_bounds_check.cpp")
    exe = str(tmp_path / "seg_bounds_check")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", "-I",
                    os.path.join(ROOT, "paper_2107_01391_amd", "csrc"), "-I", os.path.join(ROOT, "include"), src,
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "seg bounds ok" in r.stdout


# ------------------------------------------------------------ tuning table

def test_tuning_defaults_set_get_clear_and_file(tmp_path):
    d = B.key_desc("u32", base=256, ndims=4)
    B.rs_tuning_clear()
    t = B.rs_tuning_get(d, 1 << 20, True)
    assert t.tile_block in (256, 512) and 4 <= t.digit_bits <= 11
    mine = B.Tuning(4, 100, 256, 0, 12345)
    B.rs_tuning_set(d, 1 << 20, True, False, mine)
    got = B.rs_tuning_get(d, (1 << 21) - 1, True)  # same size class
    assert got.as_dict() == mine.as_dict()
    other = B.rs_tuning_get(d, 1 << 21, True)  # next class: defaults
    assert other.as_dict() == t.as_dict()
    assert B.rs_tuning_get(d, 1 << 20, False).as_dict() == t.as_dict()  # keys only: its own entry
    path = str(tmp_path / "tuning.txt")
    B.rs_tuning_save(path)
    B.rs_tuning_clear()
    assert B.rs_tuning_get(d, 1 << 20, True).as_dict() == t.as_dict()
    B.rs_tuning_load(path)
    assert B.rs_tuning_get(d, 1 << 20, True).as_dict() == mine.as_dict()
    B.rs_tuning_clear()


def test_tuning_rejects_bad_fields_and_files(tmp_path):
    d = B.key_desc("u32")
    for bad in (B.Tuning(3, 1024, 256, 0, 1), B.Tuning(8, 1, 256, 0, 1), B.Tuning(8, 1024, 300, 0, 1)):
        with pytest.raises(B.RSError) as e:
            B.rs_tuning_set(d, 1000, True, False, bad)
        assert e.value.status == 2
    p = tmp_path / "bad.txt"
    p.write_text("1 2 3\n")
    with pytest.raises(B.RSError):
        B.rs_tuning_load(str(p))


def test_tuned_choice_changes_the_plan_not_the_contract():
    """A kept choice reaches the planner: 4-bit passes need another tmp size."""
    d = B.key_desc("u32", base=2, ndims=32)
    B.rs_tuning_clear()
    n = 1 << 22
    default = B.rs_temp_bytes(d, n, True)
    B.rs_tuning_set(d, n, True, False, B.Tuning(4, 1024, 256, 0, 1 << 40))  # chained, 8 passes of 16 cells
    chained = B.rs_temp_bytes(d, n, True)
    B.rs_tuning_clear()
    assert chained != default
    assert B.rs_tune_temp_bytes(d, n, 0, True) >= max(chained, default)
    assert B.rs_tune_temp_bytes(d, n, 16, True) >= B.rs_batched_temp_bytes(d, n, 16, True)


def test_graph_capture_refuses_validation_and_null_out():
    d = B.key_desc("u32", validate=True)
    lib = B.load_library()
    h = ctypes.c_void_p(None)
    fake = ctypes.c_void_p(256)
    assert lib.rs_graph_sort(ctypes.byref(d), fake, fake, fake, fake, 10, fake, 1 << 20, ctypes.byref(h)) == 5
    assert h.value is None
    assert lib.rs_graph_sort(ctypes.byref(d), fake, fake, fake, fake, 10, fake, 1 << 20, None) == 1
    assert lib.rs_graph_destroy(None) == 0


# ------------------------------------------------------------------ server

def _cfg(**kw):
    c = dict(capacity=1 << 20, max_slots=64, max_batch=0, streams=2, mode=0, with_values=1, min_batch=0,
             batch_max_n=0)
    c.update(kw)
    return B.ServerConfig(*c.values())


@pytest.mark.parametrize("kw,status", [
    (dict(capacity=0), 2), (dict(capacity=(1 << 32) + 1), 2), (dict(max_slots=0), 2),
    (dict(streams=0), 2), (dict(streams=9), 2), (dict(mode=7), 2)])
def test_server_config_rejected(kw, status):
    d = B.key_desc("u32")
    lib = B.load_library()
    need = ctypes.c_size_t(0)
    assert lib.rs_server_work_bytes(ctypes.byref(d), ctypes.byref(_cfg(**kw)), ctypes.byref(need)) == status
    assert B.rs_last_error()


def test_server_work_bytes_and_create_checks_before_any_device_call():
    d = B.key_desc("u32")
    lib = B.load_library()
    need = ctypes.c_size_t(0)
    assert lib.rs_server_work_bytes(ctypes.byref(d), ctypes.byref(_cfg()), ctypes.byref(need)) == 0
    one = ctypes.c_size_t(0)
    assert lib.rs_server_work_bytes(ctypes.byref(d), ctypes.byref(_cfg(streams=1)), ctypes.byref(one)) == 0
    assert need.value >= 2 * one.value - 256 and one.value > 0
    per = ctypes.c_size_t(0)
    assert lib.rs_server_work_bytes(ctypes.byref(d), ctypes.byref(_cfg(mode=1)), ctypes.byref(per)) == 0
    h = ctypes.c_void_p(None)
    fake = ctypes.c_void_p(1 << 20)
    # missing arenas, then work too small, then validation refused: all before any HIP call
    assert lib.rs_server_create(ctypes.byref(d), ctypes.byref(_cfg()), None, None, None, None, fake, need.value,
                                ctypes.byref(h)) == 1
    assert lib.rs_server_create(ctypes.byref(d), ctypes.byref(_cfg()), fake, fake, fake, fake, fake, need.value - 1,
                                ctypes.byref(h)) == 4
    dv = B.key_desc("u32", validate=True)
    assert lib.rs_server_create(ctypes.byref(dv), ctypes.byref(_cfg()), fake, fake, fake, fake, fake, need.value,
                                ctypes.byref(h)) == 5
    assert h.value is None
    assert lib.rs_server_destroy(None) == 0
    t = ctypes.c_uint64(0)
    assert lib.rs_server_clock(ctypes.byref(t)) == 0 and t.value > 0


def test_large_bases_plan_one_dimension_per_pass():
    """A base above the default pass width still gets one dimension per pass
    (up to 2048 cells); above 2048 it is refused."""
    assert B.rs_temp_bytes(B.key_desc("u32", base=1000, ndims=3), 100_000, True) > 0
    assert B.rs_temp_bytes(B.key_desc("u32", base=2048, ndims=2), 100_000, True) > 0
    with pytest.raises(B.RSError) as e:
        B.rs_temp_bytes(B.key_desc("u32", base=3000, ndims=2), 100_000, True)
    assert e.value.status == 5


def test_signed_kinds_need_a_covering_space():
    assert B.rs_temp_bytes(B.key_desc("i32"), 1000, True) > 0
    assert B.rs_temp_bytes(B.key_desc("i64", base=16), 1000, True) > 0
    assert B.rs_temp_bytes(B.key_desc("i32", base=10, ndims=10), 1000, True) > 0
    for d in (B.key_desc("i32", base=10, ndims=9), B.key_desc("i64", base=256, ndims=7)):
        with pytest.raises(B.RSError) as e:
            B.rs_temp_bytes(d, 1000, True)
        assert e.value.status == 2
    # descending keys only never takes the (ascending) literal form, whose
    # scratch is the counts and starts of all 10^6 cells (8 MB)
    asc = B.rs_temp_bytes(B.key_desc("u32", base=10, ndims=6), 10**6, False)
    desc = B.rs_temp_bytes(B.key_desc("u32", base=10, ndims=6, descending=True), 10**6, False)
    assert asc >= 8 * 10**6 and desc != asc


def test_short_arrays_plan_one_workgroup():
    """Arrays of at most 4096 four- or eight-byte keys are sorted whole on
    chip: their scratch is one small control block, independent of n; one
    key more takes the passes and their alternate arrays.  16-byte strings
    always take the passes."""
    for kind, base, ndims in [("u32", 256, 4), ("u64", 10, 15), ("fixed_i64", 10, 9), ("i32", 256, 4),
                              ("i64", 16, 16), ("u32", 10, 6)]:
        d = B.key_desc(kind, base=base, ndims=ndims)
        for pairs in (True, False):
            short = {B.rs_temp_bytes(d, n, pairs) for n in (1, 17, 4095, 4096)}
            assert short == {256}, (kind, pairs, short)
            assert B.rs_temp_bytes(d, 4097, pairs) > 4097 * 4, (kind, pairs)
        dd = B.key_desc(kind, base=base, ndims=ndims, descending=True)
        assert B.rs_temp_bytes(dd, 4096, True) == 256
    s = B.key_desc("str", base=27, ndims=16)
    assert B.rs_temp_bytes(s, 100, True) > 100 * 16


def test_noalloc_sort_checks_before_any_device_call():
    """rs_sort_pairs_noalloc: n == 0 is a no-op, a NULL description is
    refused, and a sort whose scratch exceeds the static array is refused
    with RS_ERR_UNSUPPORTED before the array is looked up or anything runs."""
    d = B.key_desc("u32", base=256, ndims=4)
    lib = B.load_library()
    assert lib.rs_sort_pairs_noalloc(ctypes.byref(d), None, None, None, None, 0, None) == 0
    fake = ctypes.c_void_p(256)
    assert lib.rs_sort_pairs_noalloc(None, fake, fake, fake, fake, 10, None) == 1
    n_max = 1
    while B.rs_temp_bytes(d, n_max * 2, True) <= B.RS_NOALLOC_SCRATCH_BYTES:
        n_max *= 2
    too_big = 1 << 24
    assert B.rs_temp_bytes(d, too_big, True) > B.RS_NOALLOC_SCRATCH_BYTES
    assert lib.rs_sort_pairs_noalloc(ctypes.byref(d), fake, fake, fake, fake, too_big, None) == 5
    assert "static scratch" in B.rs_last_error()


@pytest.mark.parametrize("kind,base,ndims,n,pairs,form", [
    ("u32", 10, 6, 10**6, False, B.RS_FORM_LITERAL),      # the 10^6-cell decimal space, keys only
    ("u32", 10, 6, 10**6, True, B.RS_FORM_CHAINED),       # with values: grouped passes
    ("u32", 256, 4, 1 << 28, True, B.RS_FORM_PRESCANNED),
    ("u32", 256, 4, 4096, True, B.RS_FORM_LOCAL),
    ("u32", 1000, 2, 300_000, False, B.RS_FORM_LITERAL),  # two dimensions: 1000 rows of 1000 cells
    ("u32", 60_000, 1, 70_000, False, B.RS_FORM_LITERAL),  # one dimension: one row
])
def test_plan_inspect_forms_and_literal_layout(kind, base, ndims, n, pairs, form):
    d = B.key_desc(kind, base=base, ndims=ndims)
    info = B.rs_plan_inspect(d, n, pairs)
    assert info.form == form
    assert info.tmp_bytes == B.rs_temp_bytes(d, n, pairs)
    if form != B.RS_FORM_LITERAL:
        assert info.passes >= 1 and info.literal_cells == 0
        return
    cells = base ** ndims
    assert info.literal_cells == cells and info.passes == 0
    assert info.map_rows == (base if ndims >= 2 else 1)
    assert info.map_rows * info.map_inner == cells
    # counts, maps and starts lie inside tmp and do not overlap
    spans = sorted([(info.off_counts, cells * 4), (info.off_map_lo, info.map_rows * 4),
                    (info.off_map_hi, info.map_rows * 4), (info.off_starts, cells * 4)])
    for (a, la), (b, _) in zip(spans, spans[1:]):
        assert a + la <= b
    assert spans[-1][0] + spans[-1][1] <= info.tmp_bytes
