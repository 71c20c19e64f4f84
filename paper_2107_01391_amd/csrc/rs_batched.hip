// rs_batched.hip -- many independent arrays in one launch sequence.
//
//   1. rs_fill           clear per-array count tables and control words
//   2. rs_seg_plan       split arrays into small / large, number large tiles
//   3. rs_small_sort     small arrays sorted whole in LDS (one workgroup each)
//   4. rs_seg_histogram  every pass's cell counts of every large array
//   5. rs_cell_scan      exclusive scans of those counts, per (array, pass)
//   6. rs_rank_scatter   P segmented stable passes over all large arrays
//
// Every launch shape depends only on (total, nseg); the array boundaries are
// read on the device, so the whole sequence can be captured in a hipGraph
// once and replayed for other boundaries with the same (total, nseg).
#include <string.h>

#include "rs_internal.h"
#include "rs_seg_kernels.h"

namespace rs {

struct BatchedPlan {
  Plan digits;        // dimension groups and codecs (from the single-array planner)
  uint64_t total = 0;
  uint32_t nseg = 0;
  uint32_t tile = 4096, small_max = 4096;
  uint64_t tiles_bound = 0;
  uint32_t hist_grid = 1, small_grid = 1;
  size_t off_keys_alt = 0, off_vals_alt = 0, off_dstart = 0, off_status = 0, status_bytes = 0;
  size_t off_zero = 0, zero_bytes = 0;     // seg_hist + control words, cleared by one fill
  size_t off_seg_hist = 0, off_ctrl = 0;
  size_t off_large_ids = 0, off_tile_base = 0, off_small_ids = 0;
  uint32_t scan_cps = 1;
  size_t total_bytes = 0;
};

// control words: [0, P) tile counters, P scan counter, P+1 nlarge,
// P+2 nsmall, P+3.. scan chunk status
static rs_status make_batched_plan(const rs_key_desc *desc, uint64_t total, uint32_t nseg, bool pairs,
                                   BatchedPlan *bp, std::string *why) {
  BatchedPlan &b = *bp;
  b = BatchedPlan();
  rs_status st = make_plan(desc, 1, true, current_tuning(desc, total, pairs), &b.digits, why);
  if (st != RS_OK) return st;
  b.digits.pairs = pairs;
  b.digits.literal = false;
  if (nseg == 0) {
    *why = "nseg must be at least 1";
    return RS_ERR_BAD_DESC;
  }
  if (total >= (1ull << 40)) {
    *why = "total must be below 2^40";
    return RS_ERR_UNSUPPORTED;
  }
  const Plan &p = b.digits;
  const uint32_t kb = p.key.key_bytes;
  b.total = total;
  b.nseg = nseg;
  b.tile = kb >= 16 ? 2048 : 4096;
  b.small_max = b.tile;
  b.tiles_bound = (total + b.tile - 1) / b.tile + nseg;
  if (b.tiles_bound >= (1ull << 32)) {
    *why = "too many tiles";
    return RS_ERR_UNSUPPORTED;
  }
  const uint64_t cus = (uint64_t)cu_count();
  b.hist_grid = (uint32_t)(b.tiles_bound < cus * 4 ? b.tiles_bound : cus * 4);
  b.small_grid = (uint32_t)(nseg < cus * 8 ? nseg : cus * 8);
  b.scan_cps = (p.bins + kScanChunk - 1) / kScanChunk;
  const uint64_t row_words = (uint64_t)p.npasses * p.bins;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return at;
  };
  b.off_keys_alt = take(total * kb);
  if (pairs) b.off_vals_alt = take(total * 4);
  b.off_dstart = take(nseg * row_words * 4);
  b.status_bytes = ((size_t)p.npasses * b.tiles_bound * p.bins * 4 + 255) / 256 * 256;
  b.off_status = take(b.status_bytes);
  b.off_zero = off;
  b.off_seg_hist = take(nseg * row_words * 4);
  b.off_ctrl = take(((size_t)p.npasses + 3 + (size_t)nseg * p.npasses * b.scan_cps) * 4);
  b.zero_bytes = off - b.off_zero;
  b.off_large_ids = take((size_t)nseg * 4);
  b.off_tile_base = take(((size_t)nseg + 1) * 4);
  b.off_small_ids = take((size_t)nseg * 4);
  b.total_bytes = off;
  return RS_OK;
}

template <typename K, class Digit, int BITS>
static rs_status run_batched(const BatchedPlan &b, const Digit *digits, const void *keys_in, void *keys_out,
                             const uint32_t *vals_in, uint32_t *vals_out, const uint64_t *seg_off, void *tmp,
                             hipStream_t stream) {
  const Plan &p = b.digits;
  const bool pairs = p.pairs;
  constexpr int KPT = sizeof(K) >= 16 ? 8 : 16;
  char *base = (char *)tmp;
  uint32_t *ctrl = (uint32_t *)(base + b.off_ctrl);
  uint32_t *seg_hist = (uint32_t *)(base + b.off_seg_hist);
  uint32_t *dstart = (uint32_t *)(base + b.off_dstart);
  uint32_t *status = (uint32_t *)(base + b.off_status);
  uint32_t *large_ids = (uint32_t *)(base + b.off_large_ids);
  uint32_t *tile_base = (uint32_t *)(base + b.off_tile_base);
  uint32_t *small_ids = (uint32_t *)(base + b.off_small_ids);
  uint32_t *nlarge = ctrl + p.npasses + 1, *nsmall = ctrl + p.npasses + 2;
  const uint32_t row_words = p.npasses * p.bins;

  rs_status st = launch_fill(base + b.off_zero, b.zero_bytes, 0, stream);
  if (st != RS_OK) return st;

  SegPlanParams q{seg_off, b.nseg, b.small_max, b.tile, nlarge, large_ids, tile_base, nsmall, small_ids};
  RS_TIMED("rs_seg_plan", stream, hipLaunchKernelGGL((rs_seg_plan<1024>), dim3(1), dim3(1024), 0, stream, q));
  if ((st = check_launch("rs_seg_plan")) != RS_OK) return st;

  // small arrays: straight from the input to the output
  SmallParams<Digit> sp;
  memset(&sp, 0, sizeof sp);
  for (uint32_t i = 0; i < p.npasses; ++i) {
    sp.digit[i] = digits[i];
    sp.pass_cells[i] = p.pass_cells[i];
  }
  sp.npasses = p.npasses;
  sp.seg_off = seg_off;
  sp.small_ids = small_ids;
  sp.nsmall = nsmall;
  if (pairs)
    RS_TIMED("rs_small_sort", stream,
             hipLaunchKernelGGL((rs_small_sort<K, Digit, BITS, 256, KPT, true>), dim3(b.small_grid), dim3(256), 0,
                                stream, sp, (const K *)keys_in, (K *)keys_out, vals_in, vals_out));
  else
    RS_TIMED("rs_small_sort", stream,
             hipLaunchKernelGGL((rs_small_sort<K, Digit, BITS, 256, KPT, false>), dim3(b.small_grid), dim3(256), 0,
                                stream, sp, (const K *)keys_in, (K *)keys_out, nullptr, nullptr));
  if ((st = check_launch("rs_small_sort")) != RS_OK) return st;

  // large arrays: counts of every pass
  SegHistParams<Digit> h;
  memset(&h, 0, sizeof h);
  for (uint32_t i = 0; i < p.npasses; ++i) h.digit[i] = digits[i];
  h.npasses = p.npasses;
  h.stride = p.bins;
  h.tile = b.tile;
  h.seg_off = seg_off;
  h.tile_base = tile_base;
  h.large_ids = large_ids;
  h.nlarge = nlarge;
  h.seg_hist = seg_hist;
  h.zero = (uint4 *)status;
  h.zero16 = b.status_bytes / 16;
  const size_t lds = (size_t)row_words * 4;
  RS_TIMED("rs_seg_histogram", stream,
           hipLaunchKernelGGL((rs_seg_histogram<K, Digit, 256>), dim3(b.hist_grid), dim3(256), lds, stream, h,
                              (const K *)keys_in));
  if ((st = check_launch("rs_seg_histogram")) != RS_OK) return st;

  ScanParams s;
  s.in = seg_hist;
  s.part_stride = 0;
  s.nparts = 1;
  s.nseg = b.nseg * p.npasses;
  s.cells = p.bins;
  s.stride = p.bins;
  s.out = dstart;
  s.chunk_counter = ctrl + p.npasses;
  s.chunk_status = ctrl + p.npasses + 3;
  s.chunks_per_seg = b.scan_cps;
  s.nseg_dev = nlarge;
  s.nseg_mul = p.npasses;
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan<kScanBlock, kScanItems>), dim3(s.nseg * s.chunks_per_seg),
                              dim3(kScanBlock), 0, stream, s));
  if ((st = check_launch("rs_cell_scan")) != RS_OK) return st;

  // segmented passes over the large arrays
  const size_t kb = p.key.key_bytes;
  K *X = (K *)keys_out;
  K *Y = (K *)(base + b.off_keys_alt);
  uint32_t *XV = vals_out;
  uint32_t *YV = (uint32_t *)(base + b.off_vals_alt);
  const K *src = (const K *)keys_in;
  const uint32_t *srcv = vals_in;
  const bool odd = p.npasses % 2 == 1;
  if (odd && keys_in == keys_out) {
    if (hipMemcpyAsync(Y, keys_in, b.total * kb, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return fail(RS_ERR_HIP, "hipMemcpyAsync");
    src = Y;
  }
  if (pairs && odd && vals_in == vals_out) {
    if (hipMemcpyAsync(YV, vals_in, b.total * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return fail(RS_ERR_HIP, "hipMemcpyAsync");
    srcv = YV;
  }
  for (uint32_t i = 0; i < p.npasses; ++i) {
    const bool to_x = ((p.npasses - 1 - i) % 2) == 0;
    K *dst = to_x ? X : Y;
    uint32_t *dstv = to_x ? XV : YV;
    PassParams<Digit> pp;
    memset(&pp, 0, sizeof pp);
    pp.digit = digits[i];
    pp.bins = p.pass_cells[i];
    pp.n = b.total;
    pp.digit_start = dstart + (size_t)i * p.bins;
    pp.dstride = row_words;
    pp.status = status + (size_t)i * b.tiles_bound * p.bins;
    pp.tile_counter = ctrl + i;
    pp.seg_off = seg_off;
    pp.tile_base = tile_base;
    pp.large_ids = large_ids;
    pp.nlarge = nlarge;
    const dim3 grid((uint32_t)b.tiles_bound), blk(256);
    if (pairs)
      RS_TIMED("rs_rank_scatter", stream,
               hipLaunchKernelGGL((rs_rank_scatter<K, Digit, BITS, 256, KPT, true, true>), grid, blk, 0, stream, pp,
                                  src, dst, srcv, dstv));
    else
      RS_TIMED("rs_rank_scatter", stream,
               hipLaunchKernelGGL((rs_rank_scatter<K, Digit, BITS, 256, KPT, false, true>), grid, blk, 0, stream,
                                  pp, src, dst, nullptr, nullptr));
    if ((st = check_launch("rs_rank_scatter")) != RS_OK) return st;
    src = dst;
    srcv = dstv;
  }
  return RS_OK;
}

template <typename K, class Digit>
static rs_status batched_bits(const BatchedPlan &b, const Digit *d, const void *ki, void *ko, const uint32_t *vi,
                              uint32_t *vo, const uint64_t *off, void *tmp, hipStream_t s) {
  if constexpr (sizeof(K) >= 16) {  // strings: 27^2 = 729 cells per pass
    if (b.digits.bits != 10) return fail(RS_ERR_UNSUPPORTED, "string passes use 10-bit cells");
    return run_batched<K, Digit, 10>(b, d, ki, ko, vi, vo, off, tmp, s);
  }
  switch (b.digits.bits) {
  case 8:
    return run_batched<K, Digit, 8>(b, d, ki, ko, vi, vo, off, tmp, s);
  case 10:
    return run_batched<K, Digit, 10>(b, d, ki, ko, vi, vo, off, tmp, s);
  default:
    return run_batched<K, Digit, 11>(b, d, ki, ko, vi, vo, off, tmp, s);
  }
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_batched_temp_bytes(const rs_key_desc *desc, uint64_t total, uint32_t nseg, int with_values,
                                size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(RS_ERR_NULL_ARG, "bytes is NULL");
  BatchedPlan b;
  std::string why;
  rs_status st = make_batched_plan(desc, total, nseg, with_values != 0, &b, &why);
  if (st != RS_OK) return fail(st, why);
  *bytes = b.total_bytes;
  return RS_OK;
}

rs_status rs_sort_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                          uint32_t *vals_out, const uint64_t *d_seg_offsets, uint32_t nseg, uint64_t total, void *tmp,
                          size_t tmp_bytes, void *stream) {
  g_last_error.clear();
  if (!desc) return fail(RS_ERR_NULL_ARG, "desc is NULL");
  if (nseg == 0 || total == 0) return RS_OK;
  if (!keys_in || !keys_out || !d_seg_offsets || !tmp)
    return fail(RS_ERR_NULL_ARG, "keys_in, keys_out, d_seg_offsets and tmp are required");
  const bool pairs = vals_in != nullptr;
  if (pairs && !vals_out) return fail(RS_ERR_NULL_ARG, "vals_out is required with vals_in");
  BatchedPlan b;
  std::string why;
  rs_status st = make_batched_plan(desc, total, nseg, pairs, &b, &why);
  if (st != RS_OK) return fail(st, why);
  if (tmp_bytes < b.total_bytes)
    return fail(RS_ERR_TMP_TOO_SMALL,
                "tmp_bytes " + std::to_string(tmp_bytes) + " < " + std::to_string(b.total_bytes));
  if ((uintptr_t)tmp % 256 != 0) return fail(RS_ERR_UNSUPPORTED, "tmp must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (desc->flags & RS_FLAG_VALIDATE) {
    st = validate_keys(b.digits, keys_in, total, tmp, s);
    if (st != RS_OK) return st;
  }
  const uint32_t kb = b.digits.key.key_bytes;
  const Plan &p = b.digits;
  switch (p.mode) {
  case kModePow2:
    if (kb == 4) return batched_bits<uint32_t, DigitPow2>(b, p.p2, keys_in, keys_out, vals_in, vals_out,
                                                          d_seg_offsets, tmp, s);
    return batched_bits<uint64_t, DigitPow2>(b, p.p2, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, tmp, s);
  case kModeDiv32:
    if (kb == 4) return batched_bits<uint32_t, DigitDiv32>(b, p.d32, keys_in, keys_out, vals_in, vals_out,
                                                           d_seg_offsets, tmp, s);
    return batched_bits<uint64_t, DigitDiv32>(b, p.d32, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, tmp,
                                              s);
  case kModeDiv64:
    return batched_bits<uint64_t, DigitDiv64>(b, p.d64, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, tmp,
                                              s);
  case kModeStr16:
    return batched_bits<Str16, DigitStr16>(b, p.s16, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, tmp, s);
  }
  return fail(RS_ERR_BAD_DESC, "unknown digit mode");
}

}  // extern "C"
