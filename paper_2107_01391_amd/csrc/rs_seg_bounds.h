// rs_seg_bounds.h -- how the batched form resolves the caller's array
// bounds before any kernel reads keys: the arithmetic of rs_seg_plan, kept
// apart so that the host can check it.
//
// An array given as [lo, hi) is clamped into [0, extent) with at most
// RS_MAX_ELEMENTS keys; a large array's tiles are then cut at the scratch's
// tile bound.  Valid bounds pass unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs.h"

namespace rs {

struct SegBounds {
  uint64_t lo, len;
};

__host__ __device__ inline SegBounds resolve_segment(uint64_t lo, uint64_t hi, uint64_t extent) {
  SegBounds b;
  b.lo = lo < extent ? lo : extent;
  const uint64_t h = hi < b.lo ? b.lo : (hi < extent ? hi : extent);
  b.len = h - b.lo < RS_MAX_ELEMENTS ? h - b.lo : RS_MAX_ELEMENTS;
  return b;
}

// Tiles [first, last) of a large array that wants `want` tiles after
// `before` tiles of earlier arrays, cut at `bound`.
struct TileRange {
  uint32_t first, last;
};

__host__ __device__ inline TileRange cut_tiles(uint64_t before, uint32_t want, uint32_t bound) {
  TileRange r;
  r.first = (uint32_t)(before < bound ? before : bound);
  r.last = (uint32_t)(before + want < bound ? before + want : bound);
  return r;
}

}  // namespace rs
