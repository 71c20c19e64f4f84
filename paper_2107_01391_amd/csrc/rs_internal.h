// rs_internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "rs_plan.h"

namespace rs {

extern thread_local std::string g_last_error;

rs_status fail(rs_status st, const std::string &why);
int cu_count();
rs_status check_launch(const char *what);
// Keys aligned to their size, values to 4 bytes, tmp to 256 (null passes).
rs_status check_alignment(const KeyInfo &k, const void *ki, const void *ko, const void *vi, const void *vo,
                          const void *tmp);
rs_status launch_fill(void *p, size_t bytes, uint32_t value, hipStream_t stream);
rs_status validate_keys(const Plan &pl, const void *keys, uint64_t n, void *tmp, hipStream_t s);
// rs_sort_keys (pairs = false) / rs_sort_pairs (pairs = true) on a given
// scratch buffer: argument checks, plan, optional validation, launches.
rs_status sort_common(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                      uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream, bool pairs);
rs_status run_plan(const Plan &pl, const void *ki, void *ko, const uint32_t *vi, uint32_t *vo, void *tmp,
                   hipStream_t s);

// Kernel timing (rs_prof.h): event pairs around each launch while enabled.
bool prof_on();
void *prof_begin(const char *name, hipStream_t s);
void prof_end(void *token, hipStream_t s);
#define RS_TIMED(NAME, STREAM, LAUNCH)                                      \
  do {                                                                      \
    void *rs_tok_ = ::rs::prof_on() ? ::rs::prof_begin(NAME, STREAM) : nullptr; \
    LAUNCH;                                                                 \
    ::rs::prof_end(rs_tok_, STREAM);                                        \
  } while (0)

// Tile and digit-width choices for a description and size (`batched`: the
// segmented form over `n` keys in all): environment overrides, else the
// autotuner's cached choice for the size class, else the defaults.
Tuning current_tuning(const rs_key_desc *desc, uint64_t n, bool pairs, bool batched = false);

// Batched form: plan over arrays holding `total` keys within `extent`
// elements, and the launch sequence over arrays [seg_lo[i], seg_hi[i]).
rs_status make_batched(const rs_key_desc *desc, uint64_t total, uint64_t extent, uint32_t nseg, bool pairs,
                       Plan *p, std::string *why);
rs_status batched_run(const Plan &p, const void *ki, void *ko, const uint32_t *vi, uint32_t *vo,
                      const uint64_t *seg_lo, const uint64_t *seg_hi, void *tmp, hipStream_t s);
// Device copy by a kernel (capturable in a graph).
rs_status launch_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);

}  // namespace rs
