// rs_tune.cpp -- per (key kind, size class) tuning choices.
//
// Defaults, overridden by environment variables (read on every call, so a
// process can change them between calls):
//   RS_PRESCAN_MIN_N  single arrays from this length use prescanned passes
//   RS_DIGIT_BITS     width of a pass for power-of-two bases (4..11)
//   RS_TILE_BLOCK     threads per tile of prescanned passes (256 or 512)
//   RS_MAX_CELLS      largest count space of one pass for other bases (2..2048)
#include <stdlib.h>

#include "rs_internal.h"

namespace rs {

static uint64_t env_u64(const char *name, uint64_t dflt) {
  const char *v = getenv(name);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  unsigned long long x = strtoull(v, &end, 10);
  return (end && *end == 0) ? (uint64_t)x : dflt;
}

Tuning current_tuning(const rs_key_desc *desc, uint64_t n, bool pairs) {
  (void)desc;
  (void)n;
  (void)pairs;
  Tuning t;
  t.prescan_min_n = env_u64("RS_PRESCAN_MIN_N", t.prescan_min_n);
  const uint64_t cells = env_u64("RS_MAX_CELLS", t.max_cells);
  if (cells >= 2 && cells <= 2048) t.max_cells = (uint32_t)cells;
  const uint64_t block = env_u64("RS_TILE_BLOCK", t.tile_block);
  if (block == 256 || block == 512) t.tile_block = (uint32_t)block;
  const uint64_t bits = env_u64("RS_DIGIT_BITS", t.digit_bits);
  if (bits >= 4 && bits <= 11) t.digit_bits = (uint32_t)bits;
  return t;
}

}  // namespace rs
