// rs_tune.cpp -- per (key kind, size class) tuning choices.
#include "rs_internal.h"

namespace rs {

Tuning current_tuning(const rs_key_desc *desc, uint64_t n, bool pairs) {
  (void)desc;
  (void)n;
  (void)pairs;
  return Tuning();
}

}  // namespace rs
