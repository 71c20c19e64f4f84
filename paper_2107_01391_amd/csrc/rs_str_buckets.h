// rs_str_buckets.h -- the bucket hierarchy for base-27 strings of 16 symbols
// (Section 2.2's independent buckets, applied to the dimension groups of
// Section 3.1.1): after the passes over the four leading symbols the array
// is in order of its 27^4 leading cells, and every cell's keys form one
// contiguous bucket in input order.  Each bucket is then sorted on its own
// by the twelve remaining symbols:
//
//   rs_str_bucket_count  S[cell] for the leading four symbols (the hashing
//                        cycle of that group, eq. (1)), counted over the
//                        already ordered array with one atomic per run of
//                        equal cells in a wave's range; on the same read it
//                        marks a cell "mixed" where two neighbouring keys of
//                        the cell differ in the twelve trailing symbols
//   (the cell scan)      each bucket's start: the walk's running position
//   rs_str_bucket_sort   a bucket that is not mixed is already in order (its
//                        keys agree on every symbol, and the input order is
//                        the order of equal keys); a mixed one of at most 64
//                        keys is packed with others into the 64 lanes of a
//                        wave, ranked in registers and written back in place;
//                        a longer mixed one is listed for the batched passes
//                        over the twelve symbols
//
// A wave ranks its bucket by the twelve symbols as one 60-bit code (5 bits
// per symbol, most significant first, order-preserving because every symbol
// is below 32): rank = keys with a smaller code + keys with an equal code in
// earlier lanes (lanes hold the bucket in input order), found from one
// ballot per code bit, most significant first, stopping once no group of
// equal-so-far lanes can split any more.  That is the stable counting sort's
// placement (Section 2.3) over the 64 keys, with the cell order taken bit by
// bit.
#pragma once

#include "rs_kernels.h"

namespace rs {

// 27^4 cells of the four leading symbols.
constexpr uint32_t kStrBucketCells = 27u * 27u * 27u * 27u;
// Longest bucket a single wave sorts.
constexpr uint32_t kStrWaveBucket = 64;

// The twelve trailing symbols (positions 4..15) as a 60-bit code, 5 bits
// each, the first most significant: a symbol is its byte's low five bits,
// which maps pad (0) to 0 and 'a'..'z' to 1..26 as the passes' codec does
// (bytes outside the alphabet are invalid input: their keys' order is
// unspecified).  ~code (within 60 bits) for descending order.
__device__ __forceinline__ uint64_t str27_rest_code(const Str16 &k, bool descending) {
  uint64_t code = 0;
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    const uint32_t m = k.w[w] & 0x1f1f1f1fu;  // bytes 4w .. 4w+3, first in the low byte
    const uint32_t four = (m & 31u) << 15 | (m >> 8 & 31u) << 10 | (m >> 16 & 31u) << 5 | (m >> 24);
    code = code << 20 | four;
  }
  return descending ? (~code & ((1ull << 60) - 1)) : code;
}

// The twelve trailing symbols as their bytes' low five bits, three words:
// two keys agree on those symbols exactly when these words do.
__device__ __forceinline__ void str27_rest_words(const Str16 &k, uint32_t r[3]) {
#pragma unroll
  for (int w = 1; w < 4; ++w) r[w - 1] = k.w[w] & 0x1f1f1f1fu;
}

// The cell of the four leading symbols (bytes 0..3, the first most
// significant), each symbol as the passes' codec (DigitStr16) takes it, so
// that for any bytes it is the cell the two passes over those symbols order
// the array by; unrolled, with no per-symbol branch.  (cell ^ cx) + ca
// complements it for descending order.
__device__ __forceinline__ uint32_t str27_lead_cell(const Str16 &k, uint32_t cx, uint32_t ca) {
  const uint32_t m = k.w[0];
  uint32_t cell = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t byte = m >> (8 * j) & 0xffu, d = byte - 96u;
    cell = cell * 27u + (byte == 0u ? 0u : (d < 26u ? d : 26u));
  }
  return (cell ^ cx) + ca;
}

struct StrBucketParams {
  uint32_t lead_cx, lead_ca;  // descending complement of the leading cell
  uint64_t n;
  uint32_t *counts;       // [kStrBucketCells], zero before the count kernel
  uint8_t *mixed;         // [kStrBucketCells], zero before the count kernel
  const uint32_t *starts; // [kStrBucketCells] exclusive scan of counts
  uint64_t *list;         // buckets for the batched passes: lo[cap], then hi[cap]
  uint32_t *list_count;   // zero before the sort kernel; may exceed cap only if n does
  uint32_t list_cap;
  uint32_t descending;
};

// Bits [lo, hi) of a lane mask (lo < 64, hi <= 64).
__device__ __forceinline__ uint64_t lane_range(uint32_t lo, uint32_t hi) {
  return (hi >= 64 ? ~0ull : (1ull << hi) - 1) & (~0ull << lo);
}

// Each wave counts one contiguous range of the ordered array, U steps of 64
// keys loaded at once.  A run of equal cells is added when it ends, so a
// bucket inside one wave's range costs one atomic; the run still open at the
// end of a step carries into the next (its cell, keys so far, whether two of
// them differ, and the trailing symbols of the last key seen).
template <int BLOCK, int U = 4>
__global__ __launch_bounds__(BLOCK) void rs_str_bucket_count(const StrBucketParams q, const Str16 *__restrict__ keys) {
  constexpr uint32_t kNone = ~0u;  // no cell: the open run is empty
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (BLOCK / kWave);
  const uint64_t w = (uint64_t)blockIdx.x * (BLOCK / kWave) + threadIdx.x / kWave;
  const uint64_t a = w * q.n / waves, b = (w + 1) * q.n / waves;
  if (a >= b) return;  // uniform; the kernel has no barrier
  uint32_t oc = kNone, olen = 0, orr[3] = {0u, 0u, 0u};
  bool omix = false;
  if (a > 0) {  // the key before the range: a run of its cell continues here
    const Str16 p = keys[a - 1];
    oc = str27_lead_cell(p, q.lead_cx, q.lead_ca);
    str27_rest_words(p, orr);
  }
  for (uint64_t s0 = a; s0 < b; s0 += (uint64_t)U * kWave) {
    Str16 kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t e = s0 + (uint64_t)u * kWave + lane;
      kk[u] = e < b ? keys[e] : Str16{};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t e0 = s0 + (uint64_t)u * kWave;
      if (e0 >= b) break;  // uniform
      const bool valid = e0 + lane < b;  // a prefix of the wave
      const uint32_t c = valid ? str27_lead_cell(kk[u], q.lead_cx, q.lead_ca) : kNone;
      uint32_t r[3], pr[3];
      str27_rest_words(kk[u], r);
      uint32_t pc = __shfl_up(c, 1, kWave);
#pragma unroll
      for (int j = 0; j < 3; ++j) pr[j] = __shfl_up(r[j], 1, kWave);
      if (lane == 0) {
        pc = oc;
#pragma unroll
        for (int j = 0; j < 3; ++j) pr[j] = orr[j];
      }
      const bool same = valid && pc == c;
      const bool differs = same && (r[0] != pr[0] || r[1] != pr[1] || r[2] != pr[2]);
      const uint64_t heads = ballot(valid && !same);
      const uint64_t diffs = ballot(differs);
      const uint32_t nvalid = (uint32_t)__builtin_popcountll(ballot(valid));
      // the lanes before the first head continue the open run
      const uint32_t first = heads ? (uint32_t)__builtin_ctzll(heads) : nvalid;
      olen += first;
      omix = omix || (diffs & lane_range(0, first)) != 0;
      if (heads) {
        // the open run ends at the first head
        if (lane == 0 && olen > 0 && oc < kStrBucketCells) {
          atomicAdd(q.counts + oc, olen);
          if (omix) q.mixed[oc] = 1;  // every writer stores the same byte
        }
        // the runs that end within the step; the last one stays open
        const uint32_t last = 63u - (uint32_t)__builtin_clzll(heads);
        if (((heads >> lane) & 1u) && lane != last && c < kStrBucketCells) {
          const uint32_t end = (uint32_t)__builtin_ctzll(heads & (~0ull << (lane + 1)));
          atomicAdd(q.counts + c, end - lane);
          if (diffs & lane_range(lane, end)) q.mixed[c] = 1;
        }
        oc = __builtin_amdgcn_readlane(c, last);
        olen = nvalid - last;
        omix = (diffs & lane_range(last, nvalid)) != 0;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) orr[j] = __builtin_amdgcn_readlane(r[j], nvalid - 1);
    }
  }
  if (lane == 0 && olen > 0 && oc < kStrBucketCells) {
    atomicAdd(q.counts + oc, olen);
    if (omix) q.mixed[oc] = 1;
  }
}

template <int BLOCK, bool PAIRS, int DEPTH = 1>
__global__ __launch_bounds__(BLOCK) void rs_str_bucket_sort(const StrBucketParams q, Str16 *__restrict__ keys,
                                                            uint32_t *__restrict__ vals) {
  constexpr int WPB = BLOCK / kWave;
  // per wave and lane group: the buckets packed into its 64 lanes (start,
  // first lane, keys)
  __shared__ uint32_t slot_s[WPB][DEPTH][kWave], slot_off[WPB][DEPTH][kWave], slot_cnt[WPB][DEPTH][kWave];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  const uint64_t waves = (uint64_t)gridDim.x * WPB, w = (uint64_t)blockIdx.x * WPB + wv;
  const bool desc = q.descending != 0;
  // each wave takes one contiguous run of cells, the same number (within
  // one) for every wave, 64 cells at a time: their counts, starts and
  // marks in one load, then their buckets in cell order
  const uint32_t c_end = (uint32_t)((w + 1) * kStrBucketCells / waves);
  for (uint32_t c0 = (uint32_t)(w * kStrBucketCells / waves); c0 < c_end; c0 += kWave) {
    const uint32_t c = c0 + lane;
    const bool mine_cell = c < c_end;
    const uint32_t cnt_l = mine_cell ? q.counts[c] : 0u;
    const uint32_t s_l = mine_cell ? q.starts[c] : 0u;
    const bool mixed = mine_cell && q.mixed[c] != 0;
    const bool sane = (uint64_t)s_l + cnt_l <= q.n;  // always, for counts of this array

    // long mixed buckets: listed for the batched passes, one atomic a wave
    const uint64_t longs = ballot(sane && mixed && cnt_l > kStrWaveBucket);
    if (longs) {
      const int first = __builtin_ctzll(longs);
      uint32_t at = 0;
      if (lane == (uint32_t)first) at = atomicAdd(q.list_count, (uint32_t)__builtin_popcountll(longs));
      at = __builtin_amdgcn_readlane(at, first) + count_below(longs);
      if (((longs >> lane) & 1u) && at < q.list_cap) {
        q.list[at] = s_l;
        q.list[q.list_cap + at] = (uint64_t)s_l + cnt_l;
      }
    }

    // mixed buckets of at most 64 keys, as many at once as fit in the 64
    // lanes; DEPTH such lane groups are loaded before the first is ranked
    uint64_t todo = ballot(sane && mixed && cnt_l <= kStrWaveBucket);
    while (todo) {
      uint32_t used[DEPTH];
      uint64_t bs[DEPTH], active[DEPTH];
      uint32_t boff[DEPTH];
      Str16 k[DEPTH];
      uint32_t v[DEPTH];
      int ng = 0;
#pragma unroll
      for (int g = 0; g < DEPTH; ++g) {
        used[g] = 0;
        active[g] = 0;
        if (!todo) continue;  // uniform
        ++ng;
        uint64_t batch = 0;
        while (todo) {  // uniform: the next buckets in cell order while they fit
          const int j = __builtin_ctzll(todo);
          const uint32_t cj = __builtin_amdgcn_readlane(cnt_l, j);
          if (used[g] + cj > (uint32_t)kWave) break;
          batch |= 1ull << j;
          used[g] += cj;
          todo &= todo - 1;
        }
        // bucket i of the group takes lanes [off_i, off_i + cnt_i)
        const bool in_batch = (batch >> lane) & 1u;
        const uint32_t sz = in_batch ? cnt_l : 0u;
        const uint32_t off = wave_inclusive_scan(sz) - sz;
        const uint32_t ord = count_below(batch);
        if (in_batch) {
          slot_s[wv][g][ord] = s_l;
          slot_off[wv][g][ord] = off;
          slot_cnt[wv][g][ord] = cnt_l;
        }
        const uint32_t nb = (uint32_t)__builtin_popcountll(batch);
        uint32_t mine = 0;  // this lane's bucket: the last whose first lane is at or below it
        for (uint32_t i = 1; i < nb; ++i) mine += slot_off[wv][g][i] <= lane ? 1u : 0u;
        const bool valid = lane < used[g];
        const uint32_t bcnt = slot_cnt[wv][g][mine];
        boff[g] = slot_off[wv][g][mine];
        bs[g] = slot_s[wv][g][mine];
        active[g] = valid ? (bcnt >= 64 ? ~0ull : ((1ull << bcnt) - 1) << boff[g]) : 0ull;
        // a lane past the packed buckets loads its bucket's first key again
        // (it is in no bucket's lanes, and it stores nothing)
        const uint64_t at = bs[g] + (valid ? lane - boff[g] : 0u);
        k[g] = keys[at];
        if constexpr (PAIRS) v[g] = vals[at];
      }
#pragma unroll
      for (int g = 0; g < DEPTH; ++g) {
        if (g >= ng) break;  // uniform
        const bool valid = lane < used[g];
        const uint64_t code = str27_rest_code(k[g], desc);
        // lanes of the own bucket equal so far (eq) and smaller (lt), as
        // low and high words; only lanes of the own bucket are ever in eq,
        // so the other lanes' bits in a ballot do not matter
        uint32_t eq_l = (uint32_t)active[g], eq_h = (uint32_t)(active[g] >> 32), lt_l = 0, lt_h = 0;
        const uint32_t code_l = (uint32_t)code, code_h = (uint32_t)(code >> 32);
#pragma unroll
        for (int sym = 0; sym < 12; ++sym) {
#pragma unroll
          for (int j = 0; j < 5; ++j) {
            const int b = 59 - 5 * sym - j;
            const uint32_t word = b >= 32 ? code_h : code_l;
            // all ones where the bit is set
            const uint32_t sp = (uint32_t)((int32_t)(word << (31 - (b & 31))) >> 31);
            const uint64_t B = ballot(sp != 0);
            const uint32_t b_l = (uint32_t)B, b_h = (uint32_t)(B >> 32);
            lt_l |= eq_l & ~b_l & sp;
            lt_h |= eq_h & ~b_h & sp;
            eq_l &= ~(b_l ^ sp);
            eq_h &= ~(b_h ^ sp);
          }
          // after each symbol: stop once, within every group of lanes equal
          // so far, the bits still to come agree too (the groups can no
          // longer split, so no rank can change)
          if (sym < 11) {
            const uint64_t rest = code & ((1ull << (55 - 5 * sym)) - 1);
            const uint64_t eq = (uint64_t)eq_h << 32 | eq_l;
            const int leader = valid ? __builtin_ctzll(eq) : (int)lane;
            const uint64_t lead_rest = __shfl(rest, leader, kWave);
            if (ballot(valid && rest != lead_rest) == 0) break;
          }
        }
        const uint64_t lt = (uint64_t)lt_h << 32 | lt_l, eq = (uint64_t)eq_h << 32 | eq_l;
        const uint32_t rank = (uint32_t)__builtin_popcountll(lt) + count_below(eq);
        if (valid) {
          keys[bs[g] + rank] = k[g];
          if constexpr (PAIRS) vals[bs[g] + rank] = v[g];
        }
      }
    }
  }
}

}  // namespace rs
