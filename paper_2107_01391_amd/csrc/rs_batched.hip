// rs_batched.hip -- C ABI of the batched form (rs_sort_batched): many
// independent arrays sorted by one launch sequence (rs_segmented.h).
#include <string.h>

#include "rs_segmented.h"

namespace rs {

// The dimension groups come from the single-array planner; the segmented
// form sorts every group of every array (least significant first).
rs_status make_batched(const rs_key_desc *desc, uint64_t total, uint64_t extent, uint32_t nseg, bool pairs,
                       Plan *p, std::string *why) {
  const Tuning tune = current_tuning(desc, total, pairs, true);
  rs_status st = make_plan(desc, 1, true, tune, p, why);
  if (st != RS_OK) return st;
  p->pairs = pairs;
  p->literal = false;
  p->local = false;
  p->prescanned = false;
  st = make_seg_layout(*p, p->npasses, total, extent, nseg, true, prescan_block(tune, p->key.key_bytes, p->bits),
                       &p->seg, why);
  if (st != RS_OK) return st;
  p->total = p->seg.bytes;
  return RS_OK;
}

template <typename K, class Digit>
static rs_status batched_bits(const Plan &p, const Digit *d, const void *ki, void *ko, const uint32_t *vi,
                              uint32_t *vo, const uint64_t *lo, const uint64_t *hi, void *tmp, hipStream_t s) {
  char *base = (char *)tmp;
  void *ak = base + p.seg.off_alt_keys;
  uint32_t *av = vi ? (uint32_t *)(base + p.seg.off_alt_vals) : nullptr;
  if constexpr (sizeof(K) >= 16) {  // strings: 729 cells (base 27) or 256 (base 256) per pass
    if (p.bits == 10) return run_segmented<K, Digit, 10>(p, p.seg, d, ki, ko, vi, vo, ak, av, lo, hi, base, s);
    if (p.bits == 8) return run_segmented<K, Digit, 8>(p, p.seg, d, ki, ko, vi, vo, ak, av, lo, hi, base, s);
    return fail(RS_ERR_UNSUPPORTED, "string passes use 8- or 10-bit cells");
  }
  switch (p.bits) {
  case 8:
    return run_segmented<K, Digit, 8>(p, p.seg, d, ki, ko, vi, vo, ak, av, lo, hi, base, s);
  case 10:
    return run_segmented<K, Digit, 10>(p, p.seg, d, ki, ko, vi, vo, ak, av, lo, hi, base, s);
  default:
    return run_segmented<K, Digit, 11>(p, p.seg, d, ki, ko, vi, vo, ak, av, lo, hi, base, s);
  }
}

// Offsets of the batched form: non-decreasing, from 0 to total, every array
// at most RS_MAX_ELEMENTS keys.  Counts the violations into *bad.
static __global__ __launch_bounds__(256) void rs_validate_offsets(const uint64_t *__restrict__ off, uint32_t nseg,
                                                                  uint64_t total, uint32_t *__restrict__ bad) {
  uint32_t mine = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i <= nseg; i += (uint64_t)gridDim.x * 256) {
    const uint64_t a = off[i];
    if (i == 0 && a != 0) ++mine;
    if (i == nseg && a != total) ++mine;
    if (i < nseg) {
      const uint64_t b = off[i + 1];
      if (b < a || b - a > RS_MAX_ELEMENTS) ++mine;
    }
  }
  mine = wave_sum(mine);
  if (lane_id() == 0 && mine) atomicAdd(bad, mine);
}

static rs_status validate_offsets(const uint64_t *off, uint32_t nseg, uint64_t total, void *tmp, hipStream_t s) {
  uint32_t *bad = (uint32_t *)tmp;
  rs_status st = launch_fill(bad, 16, 0, s);
  if (st != RS_OK) return st;
  uint64_t blocks = ((uint64_t)nseg + 256) / 256;
  if (blocks > 1024) blocks = 1024;
  RS_TIMED("rs_validate", s,
           hipLaunchKernelGGL(rs_validate_offsets, dim3((uint32_t)blocks), dim3(256), 0, s, off, nseg, total, bad));
  if ((st = check_launch("rs_validate_offsets")) != RS_OK) return st;
  uint32_t h = 0;
  if (hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(RS_ERR_HIP, "validation copy");
  if (h) return fail(RS_ERR_BAD_DESC, std::to_string(h) + " invalid segment offsets");
  return RS_OK;
}

rs_status batched_run(const Plan &p, const void *ki, void *ko, const uint32_t *vi, uint32_t *vo,
                      const uint64_t *seg_lo, const uint64_t *seg_hi, void *tmp, hipStream_t s) {
  const uint32_t kb = p.key.key_bytes;
  switch (p.mode) {
  case kModePow2:
    if (kb == 4) return batched_bits<uint32_t, DigitPow2>(p, p.p2, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
    return batched_bits<uint64_t, DigitPow2>(p, p.p2, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
  case kModeDiv32:
    if (kb == 4) return batched_bits<uint32_t, DigitDiv32>(p, p.d32, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
    return batched_bits<uint64_t, DigitDiv32>(p, p.d32, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
  case kModeDiv64:
    return batched_bits<uint64_t, DigitDiv64>(p, p.d64, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
  case kModeStr16:
    return batched_bits<Str16, DigitStr16>(p, p.s16, ki, ko, vi, vo, seg_lo, seg_hi, tmp, s);
  }
  return fail(RS_ERR_BAD_DESC, "unknown digit mode");
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_batched_temp_bytes(const rs_key_desc *desc, uint64_t total, uint32_t nseg, int with_values,
                                size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(RS_ERR_NULL_ARG, "bytes is NULL");
  Plan p;
  std::string why;
  rs_status st = make_batched(desc, total, total, nseg, with_values != 0, &p, &why);
  if (st != RS_OK) return fail(st, why);
  *bytes = p.total;
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
  Plan p;
  std::string why;
  rs_status st = make_batched(desc, total, total, nseg, pairs, &p, &why);
  if (st != RS_OK) return fail(st, why);
  if (tmp_bytes < p.total)
    return fail(RS_ERR_TMP_TOO_SMALL, "tmp_bytes " + std::to_string(tmp_bytes) + " < " + std::to_string(p.total));
  if ((st = check_alignment(p.key, keys_in, keys_out, vals_in, vals_out, tmp)) != RS_OK) return st;
  if ((uintptr_t)d_seg_offsets % 8) return fail(RS_ERR_UNSUPPORTED, "d_seg_offsets must be 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (desc->flags & RS_FLAG_VALIDATE) {
    if ((st = validate_offsets(d_seg_offsets, nseg, total, tmp, s)) != RS_OK) return st;
    if ((st = validate_keys(p, keys_in, total, tmp, s)) != RS_OK) return st;
  }
  // when the arrays are short on average, most are sorted on chip and the
  // mean is their typical length
  if (total / nseg <= p.seg.small_max) p.seg.small_len = total / nseg;
  // array i is [offsets[i], offsets[i + 1])
  return batched_run(p, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, d_seg_offsets + 1, tmp, s);
}

}  // extern "C"
