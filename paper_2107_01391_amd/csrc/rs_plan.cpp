// rs_plan.cpp -- host planner (no device code).
#include "rs_plan.h"
#include "rs_internal.h"

#include <string.h>

namespace rs {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static bool mul_fits(uint64_t a, uint64_t b, uint64_t limit, uint64_t *out) {
  if (a != 0 && b > limit / a) return false;
  *out = a * b;
  return true;
}

rs_status key_info(const rs_key_desc *desc, KeyInfo *ki, std::string *why) {
  if (!desc) {
    *why = "desc is NULL";
    return RS_ERR_NULL_ARG;
  }
  memset(ki, 0, sizeof *ki);
  ki->kind = desc->kind;
  switch (desc->kind) {
  case RS_KEY_U32:
    ki->key_bytes = 4;
    ki->base = desc->base ? desc->base : 256;
    break;
  case RS_KEY_U64:
    ki->key_bytes = 8;
    ki->base = desc->base ? desc->base : 256;
    break;
  case RS_KEY_FIXED_I64:
    ki->key_bytes = 8;
    ki->base = desc->base ? desc->base : 10;
    break;
  case RS_KEY_I32:
    ki->key_bytes = 4;
    ki->base = desc->base ? desc->base : 256;
    ki->is_signed = true;
    ki->bias = 1ull << 31;
    break;
  case RS_KEY_I64:
    ki->key_bytes = 8;
    ki->base = desc->base ? desc->base : 256;
    ki->is_signed = true;
    ki->bias = 1ull << 63;
    break;
  case RS_KEY_STR:
    if (desc->str_width != 16) {
      *why = "strings: only str_width == 16 is supported";
      return RS_ERR_UNSUPPORTED;
    }
    if (desc->base && desc->base != 27 && desc->base != 256) {
      *why = "strings: base must be 27 (pad + a..z) or 256 (any byte)";
      return RS_ERR_BAD_DESC;
    }
    ki->key_bytes = 16;
    ki->base = desc->base ? desc->base : 27;
    ki->str_width = 16;
    if (desc->ndims && desc->ndims != 16) {
      *why = "strings: ndims must equal str_width";
      return RS_ERR_BAD_DESC;
    }
    ki->ndims = 16;
    break;
  default:
    *why = "unknown key kind";
    return RS_ERR_BAD_DESC;
  }
  if (ki->base < 2 || ki->base > 65536) {
    *why = "base must be in [2, 65536]";
    return RS_ERR_BAD_DESC;
  }
  ki->pow2 = (ki->base & (ki->base - 1)) == 0;
  ki->log2_base = 0;
  while ((1u << ki->log2_base) < ki->base) ++ki->log2_base;
  if (desc->kind != RS_KEY_STR) {
    const uint32_t value_bits = ki->key_bytes * 8;
    if (desc->ndims) {
      ki->ndims = desc->ndims;
    } else {  // enough digits for every value of the type (non-negative for fixed point)
      const uint32_t need_bits = desc->kind == RS_KEY_FIXED_I64 ? 63 : value_bits;
      unsigned __int128 cap = 1, lim = (unsigned __int128)1 << need_bits;
      uint32_t d = 0;
      while (cap < lim) {
        cap *= ki->base;
        ++d;
      }
      ki->ndims = d;
    }
    if (ki->ndims == 0 || ki->ndims > 64) {
      *why = "ndims must be in [1, 64]";
      return RS_ERR_BAD_DESC;
    }
    // a space wider than the key type is allowed only if its top digit is
    // still reachable (no dimension that every key has as zero beyond it)
    unsigned __int128 below_top = 1;
    for (uint32_t i = 0; i + 1 < ki->ndims; ++i) {
      below_top *= ki->base;
      if (below_top > ((unsigned __int128)1 << 64)) break;
    }
    if (below_top >= ((unsigned __int128)1 << value_bits)) {
      *why = "ndims larger than the key type can fill";
      return RS_ERR_BAD_DESC;
    }
  }
  uint64_t sp = 1;
  ki->space = 0;
  bool fits64 = true;
  for (uint32_t i = 0; i < ki->ndims; ++i)
    if (!mul_fits(sp, ki->base, UINT64_MAX, &sp)) {
      fits64 = false;
      break;
    }
  if (fits64) ki->space = sp;
  ki->space_fits32 = fits64 && sp <= (1ull << 32);
  if (ki->is_signed) {
    // every value of the type is a key: the space must cover 2^32 / 2^64
    const bool covers = ki->key_bytes == 4 ? (!fits64 || sp >= (1ull << 32)) : !fits64;
    if (!covers) {
      *why = "signed keys need b^N to cover every value of the type";
      return RS_ERR_BAD_DESC;
    }
  }
  ki->descending = (desc->flags & RS_FLAG_DESCENDING) != 0;
  return RS_OK;
}

// The passes of a plan: how the N digit dimensions are grouped (one count
// space per group, least significant group first), each group's codec, and
// the kernel variant.  Fails when some pass would not fit the kernels.
static rs_status plan_passes(const KeyInfo &k, const Tuning &tune, Plan &p, std::string *why) {
  // dimension groups, least significant first
  uint32_t dims_per_pass;
  if (k.kind == RS_KEY_STR) {
    // base 27: two characters per pass (27^2 = 729 cells, the 10-bit
    // kernels); base 256: one byte per pass (256 cells, the 8-bit kernels)
    p.mode = kModeStr16;
    dims_per_pass = k.base == 27 ? 2 : 1;
  } else if (k.pow2) {
    p.mode = kModePow2;
    if (k.log2_base > 11) {
      *why = "power-of-two base above 2^11 is not supported";
      return RS_ERR_UNSUPPORTED;
    }
    dims_per_pass = tune.digit_bits / k.log2_base;
    if (dims_per_pass == 0) dims_per_pass = 1;
  } else {
    p.mode = (k.key_bytes == 4 || k.space_fits32) ? kModeDiv32 : kModeDiv64;
    if (k.base > 2048) {
      *why = "a base above 2048 needs passes of more than 2048 cells";
      return RS_ERR_UNSUPPORTED;
    }
    dims_per_pass = 1;  // at least one dimension per pass, whatever max_cells says
    for (;;) {
      uint64_t c = 1;
      for (uint32_t i = 0; i <= dims_per_pass; ++i) c *= k.base;
      if (c > tune.max_cells || dims_per_pass + 1 > k.ndims) break;
      ++dims_per_pass;
    }
  }
  p.npasses = (k.ndims + dims_per_pass - 1) / dims_per_pass;
  if (p.npasses > (uint32_t)kMaxPasses) {
    *why = "too many passes for this description";
    return RS_ERR_UNSUPPORTED;
  }
  p.bins = 0;
  for (uint32_t i = 0; i < p.npasses; ++i) {
    const uint32_t lo = i * dims_per_pass;
    const uint32_t w = (k.ndims - lo) < dims_per_pass ? (k.ndims - lo) : dims_per_pass;
    uint64_t cells = 1, below = 1;
    for (uint32_t j = 0; j < w; ++j) cells *= k.base;
    for (uint32_t j = 0; j < lo && below <= UINT64_MAX / k.base; ++j) below *= k.base;
    p.pass_cells[i] = (uint32_t)cells;
    if (cells > p.bins) p.bins = (uint32_t)cells;
    switch (p.mode) {
    case kModePow2:
      p.p2[i].shift = lo * k.log2_base;
      p.p2[i].mask = (uint32_t)(cells - 1);
      p.p2[i].flip = k.descending ? (uint32_t)(cells - 1) : 0u;
      p.p2[i].bias = k.bias;
      break;
    case kModeDiv32:
      p.d32[i].by_lo = make_fastdiv32((uint32_t)below);
      p.d32[i].by_cells = make_fastdiv32((uint32_t)cells);
      p.d32[i].cells = (uint32_t)cells;
      p.d32[i].cx = k.descending ? ~0u : 0u;
      p.d32[i].ca = k.descending ? (uint32_t)cells : 0u;
      p.d32[i].bias = k.bias;
      break;
    case kModeDiv64:
      p.d64[i].by_lo = make_fastdiv64(below);
      p.d64[i].by_cells = make_fastdiv64(cells);
      p.d64[i].cells = (uint32_t)cells;
      p.d64[i].cx = k.descending ? ~0u : 0u;
      p.d64[i].ca = k.descending ? (uint32_t)cells : 0u;
      p.d64[i].bias = k.bias;
      break;
    case kModeStr16:
      p.s16[i].pos = k.ndims - lo - w;
      p.s16[i].width = w;
      p.s16[i].base = k.base;
      p.s16[i].cx = k.descending ? ~0u : 0u;
      p.s16[i].ca = k.descending ? (uint32_t)cells : 0u;
      break;
    }
  }
  p.bits = p.bins <= 256 ? 8 : (p.bins <= 1024 ? 10 : 11);
  if (p.bins > 2048) {
    *why = "a pass with more than 2048 cells is not supported";
    return RS_ERR_UNSUPPORTED;
  }
  if (p.mode == kModeStr16 && p.bits == 10 && p.bins > 736) {
    // the 16-byte scatter sizes its tables for base-27 symbol pairs
    *why = "string passes of more than 736 cells are not supported";
    return RS_ERR_UNSUPPORTED;
  }

  if ((size_t)p.npasses * p.bins * 4 > 64 * 1024) {
    *why = "the passes' count tables exceed 64 KiB of LDS";
    return RS_ERR_UNSUPPORTED;
  }

  return RS_OK;
}

rs_status make_plan(const rs_key_desc *desc, uint64_t n, bool pairs, const Tuning &tune, Plan *plan,
                    std::string *why) {
  Plan &p = *plan;
  p = Plan();
  rs_status st = key_info(desc, &p.key, why);
  if (st != RS_OK) return st;
  if (n > RS_MAX_ELEMENTS) {
    *why = "n exceeds RS_MAX_ELEMENTS (counts are 30-bit in the look-back words)";
    return RS_ERR_UNSUPPORTED;
  }
  const KeyInfo &k = p.key;
  p.pairs = pairs;
  p.n = n;

  // keys alone on a small integer space: the literal count / scan / emit
  if (!pairs && k.kind != RS_KEY_STR && !k.is_signed && !k.descending && k.space && k.space <= kLiteralMaxCells &&
      k.space <= (n * 4 > 65536 ? n * 4 : 65536)) {
    p.literal = true;
    p.literal_cells = (uint32_t)k.space;
    // traverse maps: one row per value of the leading coordinate
    p.map_rows = k.ndims >= 2 ? k.base : 1;
    p.map_inner = p.literal_cells / p.map_rows;
  }

  // the passes; a literal plan does not use them, so a shape the passes
  // cannot take does not stop it
  st = plan_passes(k, tune, p, why);
  if (st != RS_OK && !p.literal) return st;
  if (st != RS_OK) {
    why->clear();
    p.npasses = 0;
    p.bins = 256;
    p.bits = 8;
  } else if (n <= kLocalMaxN && k.key_bytes <= 8) {
    // a short array: every pass on chip in one workgroup, one launch
    p.local = true;
    p.literal = false;
  }

  // tile shape: 256 threads (chained), or the tuned width (prescanned);
  // keys per thread sized so that the LDS staging of one tile stays at
  // 32 KiB per 256 threads for wide keys
  p.prescanned = !p.literal && !p.local && n >= tune.prescan_min_n;
  // 8-byte keys whose space fits 32 bits (unsigned, or fixed point below
  // 10^9): narrowed once, sorted as 32-bit words, widened at the end
  p.narrow = p.prescanned && k.key_bytes == 8 && !k.is_signed && k.space && k.space <= (1ull << 32) &&
             p.npasses >= 2 && p.mode != kModeDiv64;
  p.block = p.prescanned ? prescan_block(tune, k.key_bytes, p.bits) : 256;
  p.kpt = k.key_bytes >= 16 ? 8 : 16;
  p.tile = p.block * p.kpt;
  p.ntiles = (n + p.tile - 1) / p.tile;

  // histogram grid: enough workgroups to fill 256 CUs, down to 4096 keys
  // each for small arrays
  const uint64_t words = (uint64_t)p.npasses * p.bins;
  uint64_t g = (n + 16383) / 16384;
  if (g < 256) g = (n + 4095) / 4096 < 256 ? (n + 4095) / 4096 : 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  p.hist_grid = (uint32_t)g;
  p.hist_copies = count_copies((uint32_t)words, kLdsCountBudget);

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  if (p.local) {
    p.off_ctrl = take(4);  // the validation count
  } else if (p.literal) {
    // counts and both traverse maps are contiguous: one zero fill clears
    // them; the chunk sums are written whole
    p.scan_chunks = (p.literal_cells + kBigScanChunk - 1) / kBigScanChunk;
    p.off_counts = take((size_t)p.literal_cells * 4);
    p.off_map_hi = take((size_t)p.map_rows * 4);
    p.off_map_lo = take((size_t)p.map_rows * 4);
    p.ctrl_bytes = off - p.off_counts;
    p.off_sums = take((size_t)p.scan_chunks * 4);
    p.off_starts = take((size_t)p.literal_cells * 4);
  } else if (p.prescanned) {
    // narrowed keys: two 32-bit arrays, the second 256-byte aligned
    p.off_keys_alt = take((size_t)n * k.key_bytes + (p.narrow ? 256 : 0));
    if (pairs) p.off_vals_alt = take((size_t)n * 4);
    const uint64_t entries = (uint64_t)p.bins * p.ntiles;
    p.scan_chunks = (uint32_t)((entries + kBigScanChunk - 1) / kBigScanChunk);
    p.off_table = take(entries * 4);
    uint64_t gw = 0;
    for (uint32_t i = 0; i < p.npasses; ++i) {
      const uint64_t w = group_words(p.pass_cells[i], p.ntiles);
      gw = w > gw ? w : gw;
    }
    p.off_sums = take((size_t)(gw > p.scan_chunks ? gw : p.scan_chunks) * 4);
    if (p.mode == kModeStr16 && k.base == 27 && k.ndims == 16 && p.npasses == 8 && n >= kStrBucketMinN) {
      // 27^4 buckets of the four leading symbols; at most n / 65 of them
      // hold more than 64 keys (the ones a wave cannot sort)
      const uint64_t cells = 27ull * 27 * 27 * 27;
      p.str_buckets = true;
      p.off_bcounts = take(cells * 4);
      p.off_bctrl = take(4);
      p.off_bmixed = take(cells);
      p.bfill_bytes = off - p.off_bcounts;
      p.off_bstarts = take(cells * 4);
      p.off_bsums = take((cells + kBigScanChunk - 1) / kBigScanChunk * 4);
      p.blist_cap = (uint32_t)(n / 65 + 1);
      p.off_blist = take((size_t)p.blist_cap * 16);
      rs_status sst = make_seg_layout(p, 6, n, n, p.blist_cap, false, 256, &p.bseg, why);
      if (sst != RS_OK) return sst;
      p.off_bseg = take(p.bseg.bytes);
    }
  } else {
    p.off_keys_alt = take((size_t)n * k.key_bytes);
    if (pairs) p.off_vals_alt = take((size_t)n * 4);
    p.off_dstart = take(words * 4);
    p.status_bytes = align_up((size_t)p.npasses * p.ntiles * p.bins * 4, 256);
    p.off_status = take(p.status_bytes);
    // control: [0, P) tile counters, P scan counter, P+1.. scan chunk status,
    // then the global count table [P][bins]
    p.scan_chunks = p.npasses * ((p.bins + kScanChunk - 1) / kScanChunk);
    p.off_ctrl = take(((size_t)p.npasses + 1 + p.scan_chunks + words) * 4);
    p.ctrl_bytes = off - p.off_ctrl;
  }
  p.total = off ? off : 256;
  return RS_OK;
}

// Tiles per count workgroup.  Each workgroup writes runs of TPW entries of
// the cell-major table (32 tiles of 256 cells: 128-byte runs); with `many`
// = 32 tiles per CU:
// - at most 256 cells: 32 from 2 * many tiles, 8 from many;
// - below that, 256 cells: the power of two nearest (on a log scale) to the
//   tiles that make two workgroups per CU, at most 8 (measured in the sort
//   on MI355X: 2^24 u32 pairs 408 -> 396 us with 4, 2^25 720 -> 670 us
//   with 8, against one tile each); fewer cells keep one tile each, since
//   more tiles per workgroup leave fewer LDS copies of each table and lanes
//   of a wave collide on fewer words (100 cells at 12,208 tiles: 0.153 ms
//   per pass with 32 tiles and one copy, 0.099 ms with 8 and four copies);
// - more cells: 8 from many tiles (LDS), else 1.
uint32_t tile_hist_tpw(uint32_t cells, uint64_t ntiles) {
  const uint64_t cus = (uint64_t)cu_count(), many = cus * 32;
  if (cells <= 256 && ntiles >= 2 * many) return 32;
  if (ntiles >= many) return 8;
  if (cells != 256) return 1;
  const double per = (double)ntiles / (2.0 * (double)cus);
  uint32_t tpw = 1;
  while (tpw < 8 && (double)tpw * 1.4142135623730951 < per) tpw <<= 1;
  return tpw;
}

uint64_t group_words(uint32_t cells, uint64_t ntiles) {
  const uint32_t tpw = tile_hist_tpw(cells, ntiles);
  const uint64_t rows = ((uint64_t)cells * ((ntiles + tpw - 1) / tpw) + 63) / 64 * 64;
  return tpw > 1 ? 2 * rows : rows;
}

uint32_t prescan_block(const Tuning &tune, uint32_t key_bytes, uint32_t bits) {
  return (key_bytes <= 8 && bits <= 10 && tune.tile_block == 512) ? 512u : 256u;
}

rs_status make_seg_layout(const Plan &p, uint32_t npasses, uint64_t total, uint64_t extent, uint32_t nseg,
                          bool own_alt, uint32_t block, SegLayout *Lp, std::string *why) {
  SegLayout &L = *Lp;
  L = SegLayout();
  if (nseg == 0) {
    *why = "nseg must be at least 1";
    return RS_ERR_BAD_DESC;
  }
  if (extent >= (1ull << 40) || total > extent) {
    *why = "total must be below 2^40 and within the extent";
    return RS_ERR_UNSUPPORTED;
  }
  const uint32_t kb = p.key.key_bytes;
  L.npasses = npasses;
  L.total = total;
  L.extent = extent;
  L.nseg = nseg;
  L.own_alt = own_alt;
  L.block = kb <= 8 && block == 512 ? 512 : 256;
  L.tile = L.block * (kb >= 16 ? 8 : 16);
  L.small_max = kb >= 16 ? 2048 : 4096;  // one workgroup of 256 threads sorts it in LDS
  // a large array spans more than one tile, so there are at most
  // total / tile of them, each adding at most one partial tile
  const uint64_t full = (total + L.tile - 1) / L.tile;
  L.tiles_bound = full + (nseg < total / L.tile ? nseg : total / L.tile);
  if (L.tiles_bound == 0) L.tiles_bound = 1;
  if (L.tiles_bound >= (1ull << 31)) {
    *why = "too many tiles";
    return RS_ERR_UNSUPPORTED;
  }
  const uint64_t cus = 256;
  L.small_grid = (uint32_t)(nseg < cus * 8 ? nseg : cus * 8);

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  if (own_alt) {
    L.off_alt_keys = take(extent * kb);
    if (p.pairs) L.off_alt_vals = take(extent * 4);
  }
  L.off_ctrl = take(3 * 4);
  L.off_large_ids = take((size_t)nseg * 4);
  L.off_tile_base = take(((size_t)nseg + 1) * 4);
  L.off_small_ids = take((size_t)nseg * 4);
  L.off_bounds = take((size_t)nseg * 16);
  L.off_tiles = take(L.tiles_bound * 32);
  const uint64_t entries = (uint64_t)p.bins * L.tiles_bound;
  L.off_table = take(entries * 4);
  L.off_sums = take((entries + kBigScanChunk - 1) / kBigScanChunk * 4);
  L.bytes = off;
  return RS_OK;
}

}  // namespace rs
