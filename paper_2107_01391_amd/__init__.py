"""MI355X (gfx950) Recombinant Sort.

The C ABI of ``include/rs.h`` (librs.so, hand-written HIP kernels) under the
same names, plus torch-side buffer helpers in ``api``.  Importing the package
does not load the library; the first call does, and raises ``RSError`` when
it has not been built.
"""
from ._binding import (EXPORTED, KINDS, RS_FLAG_VALIDATE, RS_KEY_FIXED_I64, RS_KEY_STR, RS_KEY_U32, RS_KEY_U64,
                       RS_MAX_ELEMENTS, KeyDesc, RSError, key_desc, load_library, rs_batched_temp_bytes,
                       rs_last_error, rs_prof_enable, rs_prof_query, rs_sort_batched, rs_sort_keys, rs_sort_pairs, rs_status_string,
                       rs_temp_bytes)

__all__ = ["EXPORTED", "KINDS", "RS_FLAG_VALIDATE", "RS_KEY_FIXED_I64", "RS_KEY_STR", "RS_KEY_U32", "RS_KEY_U64",
           "RS_MAX_ELEMENTS", "KeyDesc", "RSError", "key_desc", "load_library", "rs_batched_temp_bytes",
           "rs_last_error", "rs_prof_enable", "rs_prof_query", "rs_sort_batched", "rs_sort_keys", "rs_sort_pairs", "rs_status_string", "rs_temp_bytes"]
