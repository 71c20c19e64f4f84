// rs_plan.h -- host planner of the gfx950 Recombinant Sort path.
//
// Turns a key description into the passes of the hot path: how the N digit
// dimensions are grouped (one count space per group), which codec extracts a
// group's cell, the order of the passes, the tile shape of the kernels, and
// the layout of the caller's scratch buffer.
//
// A single array is sorted in one of three ways:
//   literal     keys alone on a small integer space: the whole space is one
//               count space (count, scan, emit rebuilt keys);
//   chained     stable passes over the groups, least significant first, each
//               pass one kernel whose tiles chain their offsets by look-back
//               (few launches: small arrays);
//   prescanned  the same passes, each as per-tile counts, one flat scan and
//               a scatter whose offsets are read from the scanned table (no
//               chain between tiles: large arrays).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "rs.h"
#include "rs_device.h"

namespace rs {

enum DigitMode { kModePow2 = 0, kModeDiv32 = 1, kModeDiv64 = 2, kModeStr16 = 3 };

struct KeyInfo {
  uint32_t kind, base, ndims, key_bytes, str_width;
  bool pow2;
  uint32_t log2_base;
  bool space_fits32;    // b^N <= 2^32
  uint64_t space;       // b^N when it fits 64 bits, else 0
  uint64_t bias;        // added before the digits are taken: 2^31 / 2^63 for signed keys
  bool is_signed;       // RS_KEY_I32 / RS_KEY_I64
  bool descending;      // RS_FLAG_DESCENDING
};

struct Tuning {
  uint32_t digit_bits = 8;       // target width of a pass (power-of-two bases)
  uint32_t max_cells = 256;      // largest count space of one pass (other bases; strings: 729)
  uint64_t prescan_min_n = 1ull << 21;  // single arrays from this size use prescanned passes
  uint32_t tile_block = 512;            // threads per tile of prescanned passes (256 or 512)
};

// Scratch layout of the segmented form over `nseg` arrays holding `total`
// keys, sorted by passes [0, npasses) of a parent plan (least significant
// first).  Offsets are relative to the start of the segmented region.
struct SegLayout {
  uint32_t npasses = 0;
  uint64_t total = 0;   // keys in all arrays
  uint64_t extent = 0;  // elements the arrays span (alternate arrays' size)
  uint32_t nseg = 0;
  uint32_t block = 256, tile = 4096, small_max = 4096;
  uint64_t tiles_bound = 0;  // large-array tiles, at most
  uint32_t small_grid = 1;
  bool own_alt = false;
  bool any_large = true;  // false when the caller knows every array is small: no passes are launched
  uint64_t small_len = 0;  // typical length of the small arrays when the caller knows it, else 0
  size_t off_alt_keys = 0, off_alt_vals = 0;
  size_t off_ctrl = 0;  // nlarge, nsmall, tiles in use
  size_t off_large_ids = 0, off_tile_base = 0, off_small_ids = 0;
  size_t off_bounds = 0;  // resolved array bounds: lo[nseg], then hi[nseg]
  size_t off_tiles = 0;  // TileDesc per tile id
  size_t off_table = 0, off_sums = 0;  // per-tile count table and its chunk sums
  size_t bytes = 0;
};

struct Plan {
  KeyInfo key;
  bool pairs = false;
  bool literal = false;      // keys only, whole space counted at once
  bool local = false;        // short array: one workgroup sorts it on chip
  bool narrow = false;       // 8-byte keys below 2^32: the passes move them as 32-bit words
  uint32_t literal_cells = 0;
  uint32_t map_rows = 1, map_inner = 0;  // literal: traverse-map rows and cells per row
  bool prescanned = false;   // passes without look-back

  DigitMode mode = kModePow2;
  uint32_t npasses = 0;      // passes in least-significant-first order
  uint32_t bins = 0;         // cells of the widest pass
  uint32_t bits = 8;         // kernel variant: 8, 10 or 11 bits of cell index
  uint32_t pass_cells[kMaxPasses] = {};
  DigitPow2 p2[kMaxPasses] = {};
  DigitDiv32 d32[kMaxPasses] = {};
  DigitDiv64 d64[kMaxPasses] = {};
  DigitStr16 s16[kMaxPasses] = {};

  uint32_t block = 256, kpt = 16, tile = 4096;
  uint64_t n = 0, ntiles = 0;
  uint32_t hist_grid = 1, hist_copies = 1;

  // scratch layout (byte offsets into tmp)
  size_t off_keys_alt = 0, off_vals_alt = 0, off_dstart = 0, off_status = 0;
  size_t off_ctrl = 0, ctrl_bytes = 0, status_bytes = 0;
  size_t off_counts = 0, off_starts = 0;
  size_t off_map_lo = 0, off_map_hi = 0;  // literal: traverse maps (complemented minima, maxima)
  // prescanned: per-tile counts, and at off_sums what the count kernel
  // leaves for the scan (group_words)
  size_t off_table = 0, off_sums = 0;
  uint32_t scan_chunks = 0;            // chunks of the cell scan
  SegLayout seg;                       // batched form
  // base-27 16-symbol strings, prescanned: the passes over the four leading
  // symbols, then every bucket of equal leading symbols sorted on its own
  // (rs_str_buckets.h); long buckets whose keys differ go through the
  // batched passes over the other twelve symbols (layout bseg, sized for
  // blist_cap buckets, at off_bseg; it reuses the alternate arrays)
  bool str_buckets = false;
  size_t off_bcounts = 0, off_bctrl = 0, off_bmixed = 0, off_bstarts = 0, off_bsums = 0, off_blist = 0,
         off_bseg = 0;
  size_t bfill_bytes = 0;              // counts, control word and mixed marks, cleared together
  uint32_t blist_cap = 0;
  SegLayout bseg;
  size_t total = 0;
};

rs_status key_info(const rs_key_desc *desc, KeyInfo *ki, std::string *why);
rs_status make_plan(const rs_key_desc *desc, uint64_t n, bool pairs, const Tuning &tune, Plan *plan,
                    std::string *why);
// Threads per tile of prescanned passes for keys of `key_bytes` and passes
// of kernel variant `bits` (the choice with_block() makes on the device side).
uint32_t prescan_block(const Tuning &tune, uint32_t key_bytes, uint32_t bits);
// Tiles per workgroup of the per-tile count kernel for `cells` cells over
// `ntiles` tiles (1, 8 or 32; from the device's CU count).
uint32_t tile_hist_tpw(uint32_t cells, uint64_t ntiles);
// Words the count kernel of one pass leaves for the scan of one array's
// table: per cell and workgroup its counts of the cells below, and with
// several tiles per workgroup also its total.
uint64_t group_words(uint32_t cells, uint64_t ntiles);
// Layout of the segmented form for passes [0, npasses) of `p`.
rs_status make_seg_layout(const Plan &p, uint32_t npasses, uint64_t total, uint64_t extent, uint32_t nseg,
                          bool own_alt, uint32_t block, SegLayout *L, std::string *why);

constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanItems = 8;
constexpr uint32_t kScanChunk = kScanBlock * kScanItems;
constexpr uint32_t kBigScanItems = 16;
constexpr uint32_t kBigScanChunk = kScanBlock * kBigScanItems;
constexpr uint32_t kLiteralMaxCells = 1u << 24;
// Longest array one workgroup sorts whole on chip (256 threads x 16 keys).
constexpr uint64_t kLocalMaxN = 4096;
// Base-27 strings from this many keys sort by buckets of their four leading
// symbols (fewer passes over HBM); shorter arrays run all eight passes.
constexpr uint64_t kStrBucketMinN = 1ull << 20;

}  // namespace rs
