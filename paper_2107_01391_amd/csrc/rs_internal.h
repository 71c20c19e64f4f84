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
rs_status launch_fill(void *p, size_t bytes, uint32_t value, hipStream_t stream);
rs_status validate_keys(const Plan &pl, const void *keys, uint64_t n, void *tmp, hipStream_t s);
rs_status run_plan(const Plan &pl, const void *ki, void *ko, const uint32_t *vi, uint32_t *vo, void *tmp,
                   hipStream_t s);

// Tile and digit-width choices for a description and size: the autotuner's
// cached choice when one exists, else the defaults.
Tuning current_tuning(const rs_key_desc *desc, uint64_t n, bool pairs);

}  // namespace rs
