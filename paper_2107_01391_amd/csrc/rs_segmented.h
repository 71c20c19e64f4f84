// rs_segmented.h -- launch sequence of the batched form: many independent
// arrays (bucket sort's independent buckets, Section 2.2) in one sequence.
//
//   1. rs_seg_plan       split arrays into small / large, number large tiles
//   2. rs_seg_tiles      resolve every large-array tile once
//   3. rs_small_sort / rs_local_sort
//                        small arrays sorted whole in LDS (one workgroup each)
//   4. per pass over the large arrays: rs_tile_histogram, one scan of the
//      table, rs_rank_scatter (rs_passes.h)
//
// Every launch shape depends only on (total, nseg); the array boundaries are
// read on the device, so the sequence can be captured in a hipGraph.
#pragma once

#include <string.h>

#include "rs_passes.h"
#include "rs_seg_kernels.h"

namespace rs {

// Sorts arrays [seg_lo[i], seg_hi[i]) of keys_in by passes [0, L.npasses)
// of plan p (least significant first) into the same positions of keys_out.
// The arrays lie within the first L.extent elements and do not overlap;
// alt_* are scratch arrays of L.extent elements.
// Typical small-array length up to which rs_local_sort is used.
constexpr uint64_t kLocalSortMaxLen = 2048;

template <typename K, class Digit, int BITS>
rs_status run_segmented(const Plan &p, const SegLayout &L, const Digit *digits, const void *keys_in,
                        void *keys_out, const uint32_t *vals_in, uint32_t *vals_out, void *alt_keys,
                        uint32_t *alt_vals, const uint64_t *seg_lo, const uint64_t *seg_hi, char *base,
                        hipStream_t stream) {
  const bool pairs = vals_in != nullptr;
  const uint32_t P = L.npasses;
  constexpr int KPT = sizeof(K) >= 16 ? 8 : 16;
  uint32_t *ctrl = (uint32_t *)(base + L.off_ctrl);
  uint32_t *nlarge = ctrl, *nsmall = ctrl + 1, *ntotal = ctrl + 2;
  uint32_t *large_ids = (uint32_t *)(base + L.off_large_ids);
  uint32_t *tile_base = (uint32_t *)(base + L.off_tile_base);
  uint32_t *small_ids = (uint32_t *)(base + L.off_small_ids);
  TileDesc *tiles = (TileDesc *)(base + L.off_tiles);
  uint32_t *table = (uint32_t *)(base + L.off_table);
  uint32_t *sums = (uint32_t *)(base + L.off_sums);
  rs_status st;

  // the caller's bounds are read once, by rs_seg_plan; every later kernel
  // reads the resolved (clamped) copy
  uint64_t *rlo = (uint64_t *)(base + L.off_bounds), *rhi = rlo + L.nseg;
  SegPlanParams q{seg_lo, seg_hi, L.nseg, L.small_max, L.tile, L.extent, (uint32_t)L.tiles_bound,
                  nlarge, large_ids, tile_base, nsmall, small_ids, rlo, rhi};
  RS_TIMED("rs_seg_plan", stream, hipLaunchKernelGGL((rs_seg_plan<1024>), dim3(1), dim3(1024), 0, stream, q));
  if ((st = check_launch("rs_seg_plan")) != RS_OK) return st;
  seg_lo = rlo;
  seg_hi = rhi;
  if (L.any_large) {
    SegTilesParams tq{seg_lo, seg_hi, large_ids, tile_base, nlarge, L.tile, tiles, ntotal};
    RS_TIMED("rs_seg_tiles", stream,
             hipLaunchKernelGGL(rs_seg_tiles, dim3((uint32_t)((L.tiles_bound + 255) / 256)), dim3(256), 0, stream,
                                tq));
    if ((st = check_launch("rs_seg_tiles")) != RS_OK) return st;
  }

  // small arrays: straight from the input to the output
  SmallParams<Digit> sp;
  memset(&sp, 0, sizeof sp);
  for (uint32_t i = 0; i < P; ++i) {
    sp.digit[i] = digits[i];
    sp.pass_cells[i] = p.pass_cells[i];
  }
  sp.npasses = P;
  sp.seg_lo = seg_lo;
  sp.seg_hi = seg_hi;
  sp.small_ids = small_ids;
  sp.nsmall = nsmall;
  bool launched = false;
  if constexpr (sizeof(K) <= 8) {
    // several passes over short arrays: 4-bit sub-passes with per-thread
    // counts; one pass, or arrays near the 4096-key limit, are cheaper
    // ranked by ballots (whose per-pass cell scan costs the same for any
    // length)
    if (P >= 2 && (L.small_len == 0 || L.small_len <= kLocalSortMaxLen)) {
      if (pairs)
        RS_TIMED("rs_small_sort", stream,
                 hipLaunchKernelGGL((rs_local_sort<K, Digit, 256, 16, true>), dim3(L.small_grid), dim3(256), 0,
                                    stream, sp, (const K *)keys_in, (K *)keys_out, vals_in, vals_out));
      else
        RS_TIMED("rs_small_sort", stream,
                 hipLaunchKernelGGL((rs_local_sort<K, Digit, 256, 16, false>), dim3(L.small_grid), dim3(256), 0,
                                    stream, sp, (const K *)keys_in, (K *)keys_out, nullptr, nullptr));
      launched = true;
    }
  }
  if (!launched) {
    if (pairs)
      RS_TIMED("rs_small_sort", stream,
               hipLaunchKernelGGL((rs_small_sort<K, Digit, BITS, 256, KPT, true>), dim3(L.small_grid), dim3(256), 0,
                                  stream, sp, (const K *)keys_in, (K *)keys_out, vals_in, vals_out));
    else
      RS_TIMED("rs_small_sort", stream,
               hipLaunchKernelGGL((rs_small_sort<K, Digit, BITS, 256, KPT, false>), dim3(L.small_grid), dim3(256), 0,
                                  stream, sp, (const K *)keys_in, (K *)keys_out, nullptr, nullptr));
  }
  if ((st = check_launch("rs_small_sort")) != RS_OK) return st;

  // large arrays: the passes, every array sharing each launch
  if (!L.any_large) return RS_OK;
  return with_block<K, BITS>(L.block, [&]<int BLOCK>() {
    return prescanned_passes<K, Digit, BITS, BLOCK, true>(p, digits, P, keys_in, keys_out, vals_in, vals_out,
                                                          alt_keys, alt_vals, L.extent, L.tiles_bound, table, sums,
                                                          tiles, ntotal, stream);
  });
}

}  // namespace rs
