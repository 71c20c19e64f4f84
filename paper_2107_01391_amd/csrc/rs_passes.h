// rs_passes.h -- launch sequence of one prescanned pass (reduce-then-scan):
//
//   rs_tile_histogram   per-tile counts of the pass's cells, flat table
//   (scan)              one exclusive scan of the whole table: for one
//                       array rs_group_scan (one launch; the count kernel
//                       has already summed each workgroup's tiles), for
//                       many arrays rs_cell_scan_reduce/_spine/_down
//   rs_rank_scatter     stable scatter with offsets read from the table
//
// No tile waits on another: on MI355X every serialised global round trip
// inside a tile costs the latency of a saturated HBM queue, so passes avoid
// chains between tiles entirely.  The same sequence serves one array and
// many arrays (SEG), whose tables are laid out so that one scan covers all.
#pragma once

#include <string.h>

#include "rs_internal.h"
#include "rs_kernels.h"

namespace rs {

// LDS of the per-tile count tables: two lane-group copies of eight 256-cell
// tables, small enough for eight workgroups per CU
constexpr uint32_t kTileHistBudget = 24 * 1024;

// Keys are read as KI and written as KO (narrowed on a first pass, widened
// on a last one; see rs_rank_scatter).
// For one array (SEG false), `sums` is the region the plan sizes with
// group_words: the workgroup totals of the count kernel (with several tiles
// per workgroup), then each workgroup's counts of the cells below each
// cell; for many arrays it holds the chunk sums of the three-launch scan.
template <typename K, class Digit, int BITS, int BLOCK, bool SEG, typename KI = K, typename KO = K>
rs_status prescanned_pass(const Digit &digit, uint32_t cells, bool pairs, const KI *src, KO *dst,
                          const uint32_t *srcv, uint32_t *dstv, uint64_t n, uint64_t ntiles_bound,
                          uint32_t *table, uint32_t *sums, const TileDesc *tiles, const uint32_t *ntotal,
                          hipStream_t stream) {
  constexpr int KPT = sizeof(K) >= 16 ? 8 : 16;  // LDS staging: 32 KiB per 256 threads
  constexpr int TILE = BLOCK * KPT;
  rs_status st;
  const uint64_t count = (uint64_t)cells * ntiles_bound;
  const uint32_t nchunks = (uint32_t)((count + kBigScanChunk - 1) / kBigScanChunk);
  const uint32_t tpw = tile_hist_tpw(cells, ntiles_bound);
  // one array: rows of workgroup totals (several tiles per workgroup) or of
  // the table itself (one tile per workgroup), and the workgroups' counts
  // below each cell, for rs_group_scan
  const uint64_t ngroups = (ntiles_bound + tpw - 1) / tpw;
  const uint64_t rows_words = (uint64_t)cells * ngroups;
  uint32_t *groups = tpw > 1 ? sums : nullptr;
  uint32_t *below = tpw > 1 ? sums + (rows_words + 63) / 64 * 64 : sums;

  TileHistParams<Digit> th;
  memset(&th, 0, sizeof th);
  th.digit = digit;
  th.cells = cells;
  th.ntiles = (uint32_t)ntiles_bound;
  th.n = n;
  th.counts = table;
  th.tiles = tiles;
  th.ntotal = ntotal;
  if constexpr (!SEG) {
    th.groups = groups;
    th.before = below;
    th.ngroups = ngroups;
  }
  auto histogram = [&]<int TPW>() {
    th.copies = count_copies(cells * TPW, kTileHistBudget);
    const size_t lds = (size_t)TPW * th.copies * (cells + 1) * 4;
    RS_TIMED("rs_tile_histogram", stream,
             hipLaunchKernelGGL((rs_tile_histogram<KI, Digit, 256, TPW, TILE, SEG>),
                                dim3((uint32_t)((ntiles_bound + TPW - 1) / TPW)), dim3(256), lds, stream, th, src));
  };
  switch (tpw) {
  case 32: histogram.template operator()<32>(); break;
  case 8: histogram.template operator()<8>(); break;
  case 4: histogram.template operator()<4>(); break;
  case 2: histogram.template operator()<2>(); break;
  default: histogram.template operator()<1>(); break;
  }
  if ((st = check_launch("rs_tile_histogram")) != RS_OK) return st;

  if constexpr (SEG) {
    const uint32_t *cdev = ntotal;
    RowMaps nomaps;
    memset(&nomaps, 0, sizeof nomaps);
    RS_TIMED("rs_cell_scan", stream,
             hipLaunchKernelGGL((rs_cell_scan_reduce<kScanBlock, kBigScanItems>), dim3(nchunks), dim3(kScanBlock), 0,
                                stream, table, count, cdev, cells, sums, nomaps));
    RS_TIMED("rs_cell_scan", stream,
             hipLaunchKernelGGL((rs_cell_scan_spine<1024, kBigScanChunk>), dim3(1), dim3(1024), 0, stream, sums,
                                count, cdev, cells));
    RS_TIMED("rs_cell_scan", stream,
             hipLaunchKernelGGL((rs_cell_scan_down<kScanBlock, kBigScanItems>), dim3(nchunks), dim3(kScanBlock), 0,
                                stream, table, count, cdev, cells, sums, table, nomaps));
  } else {
    constexpr uint32_t kSegTiles = kScanBlock * 16;
    GroupScanParams gs;
    gs.table = table;
    gs.groups = groups;
    gs.before = below;
    gs.ntiles = ntiles_bound;
    gs.ngroups = ngroups;
    gs.shift = (uint32_t)__builtin_ctz(tpw);
    gs.cells = cells;
    gs.segs = groups ? (uint32_t)((ntiles_bound + kSegTiles - 1) / kSegTiles) : 1u;
    RS_TIMED("rs_cell_scan", stream,
             hipLaunchKernelGGL((rs_group_scan<kScanBlock, 16>), dim3(cells * gs.segs), dim3(kScanBlock), 0, stream,
                                gs));
  }
  if ((st = check_launch("rs_cell_scan")) != RS_OK) return st;

  PassParams<Digit> pp;
  memset(&pp, 0, sizeof pp);
  pp.digit = digit;
  pp.bins = cells;
  pp.n = n;
  pp.ntiles = (uint32_t)ntiles_bound;
  pp.tile_offsets = table;
  pp.tiles = tiles;
  pp.ntotal = ntotal;
  constexpr int MODE = SEG ? kPrescannedSeg : kPrescanned;
  const dim3 grid((uint32_t)((ntiles_bound + 7) / 8 * 8)), blk(BLOCK);
  if (pairs)
    RS_TIMED("rs_rank_scatter", stream,
             hipLaunchKernelGGL((rs_rank_scatter<K, Digit, BITS, BLOCK, KPT, true, MODE, KI, KO>), grid, blk, 0,
                                stream, pp, src, dst, srcv, dstv));
  else
    RS_TIMED("rs_rank_scatter", stream,
             hipLaunchKernelGGL((rs_rank_scatter<K, Digit, BITS, BLOCK, KPT, false, MODE, KI, KO>), grid, blk, 0,
                                stream, pp, src, dst, nullptr, nullptr));
  return check_launch("rs_rank_scatter");
}

// Calls f.template operator()<BLOCK>() with the plan's tile width: 512
// threads (8192 keys per tile) or 256.  Wide tiles make each cell's run of
// output per tile longer, so fewer output lines are written in part; keys
// of 16 bytes keep 256 threads (LDS staging).
template <typename K, int BITS, class F>
rs_status with_block(uint32_t block, F &&f) {
  if constexpr (sizeof(K) <= 8 && BITS <= 10) {
    if (block == 512) return f.template operator()<512>();
  }
  return f.template operator()<256>();
}

// Runs passes [0, P) (least significant first) from keys_in to keys_out,
// ping-ponging through alt; the last pass writes keys_out.  When the input
// is the output and P is odd, the input is first copied to alt.
template <typename K, class Digit, int BITS, int BLOCK, bool SEG>
rs_status prescanned_passes(const Plan &p, const Digit *digits, uint32_t P, const void *keys_in, void *keys_out,
                            const uint32_t *vals_in, uint32_t *vals_out, void *alt_keys, uint32_t *alt_vals,
                            uint64_t n, uint64_t ntiles_bound, uint32_t *table, uint32_t *sums,
                            const TileDesc *tiles, const uint32_t *ntotal, hipStream_t stream) {
  const bool pairs = vals_in != nullptr;
  K *X = (K *)keys_out;
  K *Y = (K *)alt_keys;
  uint32_t *XV = vals_out;
  uint32_t *YV = alt_vals;
  const K *src = (const K *)keys_in;
  const uint32_t *srcv = vals_in;
  const bool odd = P % 2 == 1;
  rs_status st;
  if (odd && keys_in == keys_out) {
    if ((st = launch_copy(Y, keys_in, n * p.key.key_bytes, stream)) != RS_OK) return st;
    src = Y;
  }
  if (pairs && odd && vals_in == vals_out) {
    if ((st = launch_copy(YV, vals_in, n * 4, stream)) != RS_OK) return st;
    srcv = YV;
  }
  for (uint32_t i = 0; i < P; ++i) {
    const bool to_x = ((P - 1 - i) % 2) == 0;
    K *dst = to_x ? X : Y;
    uint32_t *dstv = to_x ? XV : YV;
    st = prescanned_pass<K, Digit, BITS, BLOCK, SEG>(digits[i], p.pass_cells[i], pairs, src, dst, srcv,
                                                                dstv, n, ntiles_bound, table, sums, tiles, ntotal,
                                                                stream);
    if (st != RS_OK) return st;
    src = dst;
    srcv = dstv;
  }
  return RS_OK;
}

// Passes [0, P) over 8-byte keys whose space fits 32 bits, moved as 32-bit
// words in between: the first pass reads the 8-byte input and writes 32-bit
// words to a, the middle passes ping-pong between a and b, the last pass
// writes the 8-byte output (zero-extended).  P >= 2.  Values ping-pong
// between vals_out and alt_vals as in prescanned_passes.
template <class Digit, int BITS, int BLOCK>
rs_status narrowed_passes(const Plan &p, const Digit *digits, uint32_t P, const uint64_t *keys_in,
                          uint64_t *keys_out, const uint32_t *vals_in, uint32_t *vals_out, uint32_t *a,
                          uint32_t *b, uint32_t *alt_vals, uint64_t n, uint64_t ntiles_bound, uint32_t *table,
                          uint32_t *sums, hipStream_t stream) {
  const bool pairs = vals_in != nullptr;
  uint32_t *XV = vals_out, *YV = alt_vals;
  const uint32_t *srcv = vals_in;
  rs_status st;
  if (pairs && P % 2 == 1 && vals_in == vals_out) {
    if ((st = launch_copy(YV, vals_in, n * 4, stream)) != RS_OK) return st;
    srcv = YV;
  }
  const uint32_t *ksrc = nullptr;  // the 32-bit words of the previous pass
  for (uint32_t i = 0; i < P; ++i) {
    const bool to_x = ((P - 1 - i) % 2) == 0;
    uint32_t *dstv = to_x ? XV : YV;
    uint32_t *kdst = i % 2 == 0 ? a : b;
    if (i == 0)
      st = prescanned_pass<uint32_t, Digit, BITS, BLOCK, false, uint64_t, uint32_t>(
          digits[i], p.pass_cells[i], pairs, keys_in, kdst, srcv, dstv, n, ntiles_bound, table, sums, nullptr,
          nullptr, stream);
    else if (i + 1 == P)
      st = prescanned_pass<uint32_t, Digit, BITS, BLOCK, false, uint32_t, uint64_t>(
          digits[i], p.pass_cells[i], pairs, ksrc, keys_out, srcv, dstv, n, ntiles_bound, table, sums, nullptr,
          nullptr, stream);
    else
      st = prescanned_pass<uint32_t, Digit, BITS, BLOCK, false>(digits[i], p.pass_cells[i], pairs, ksrc, kdst, srcv,
                                                                  dstv, n, ntiles_bound, table, sums, nullptr,
                                                                  nullptr, stream);
    if (st != RS_OK) return st;
    ksrc = kdst;
    srcv = dstv;
  }
  return RS_OK;
}

}  // namespace rs
