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
//                        equal cells in a wave
//   (the cell scan)      each bucket's start: the walk's running position
//   rs_str_bucket_sort   buckets of at most 64 keys packed into the 64 lanes
//                        of a wave, ranked in registers and written back in
//                        place; a longer bucket whose keys agree on all
//                        twelve symbols is already in order; any other is
//                        listed for the batched passes over the twelve
//                        symbols
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

struct StrBucketParams {
  DigitStr16 lead;        // cell of the four leading symbols, as the passes order them
  uint64_t n;
  uint32_t *counts;       // [kStrBucketCells], zero before the count kernel
  const uint32_t *starts; // [kStrBucketCells] exclusive scan of counts
  uint64_t *list;         // buckets for the batched passes: lo[cap], then hi[cap]
  uint32_t *list_count;   // zero before the sort kernel; may exceed cap only if n does
  uint32_t list_cap;
  uint32_t descending;
};

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_str_bucket_count(const StrBucketParams q, const Str16 *__restrict__ keys) {
  const uint32_t lane = lane_id();
  for (uint64_t base = (uint64_t)blockIdx.x * BLOCK; base < q.n; base += (uint64_t)gridDim.x * BLOCK) {
    const uint64_t e = base + threadIdx.x;
    const bool valid = e < q.n;
    const uint32_t c = valid ? q.lead(keys[e]) : 0u;
    const uint32_t prev = __shfl_up(c, 1, kWave);
    const bool head = valid && (lane == 0 || prev != c);
    const uint64_t heads = ballot(head);
    const uint64_t live = ballot(valid);
    if (head) {
      // the run ends at the next head, or at the wave's last valid lane
      const uint64_t later = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
      const uint32_t end = later ? (uint32_t)__builtin_ctzll(later) : 64u - (uint32_t)__builtin_clzll(live);
      if (c < kStrBucketCells) atomicAdd(q.counts + c, end - lane);
    }
  }
}

template <int BLOCK, bool PAIRS, int DEPTH = 1, int CHUNK = 64>
__global__ __launch_bounds__(BLOCK) void rs_str_bucket_sort(const StrBucketParams q, Str16 *__restrict__ keys,
                                                            uint32_t *__restrict__ vals) {
  constexpr int WPB = BLOCK / kWave;
  // per wave and lane group: the buckets packed into its 64 lanes (start,
  // first lane, keys)
  __shared__ uint32_t slot_s[WPB][DEPTH][kWave], slot_off[WPB][DEPTH][kWave], slot_cnt[WPB][DEPTH][kWave];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  const uint32_t waves = gridDim.x * WPB;
  const bool desc = q.descending != 0;
  // each wave takes CHUNK cells at a time (small steps balance the waves'
  // work): their counts and starts in one load, then their buckets in cell
  // order
  static_assert(CHUNK <= kWave, "one cell per lane");
  for (uint32_t c0 = (blockIdx.x * WPB + wv) * CHUNK; c0 < kStrBucketCells; c0 += waves * CHUNK) {
    const uint32_t c = c0 + lane;
    const bool mine_cell = lane < (uint32_t)CHUNK && c < kStrBucketCells;
    const uint32_t cnt_l = mine_cell ? q.counts[c] : 0u;
    const uint32_t s_l = mine_cell ? q.starts[c] : 0u;
    const bool sane = (uint64_t)s_l + cnt_l <= q.n;  // always, for counts of this array

    // long buckets: already in order when their keys agree on the twelve
    // symbols (the input order is the order of equal keys); else listed
    uint64_t longs = ballot(sane && cnt_l > kStrWaveBucket);
    while (longs) {
      const int j = __builtin_ctzll(longs);
      longs &= longs - 1;
      const uint32_t cnt = __builtin_amdgcn_readlane(cnt_l, j);
      const uint64_t s = __builtin_amdgcn_readlane(s_l, j);
      uint64_t lo = ~0ull, hi = 0;
      constexpr uint32_t U = 16;  // loads in flight per lane
      for (uint32_t i0 = 0; i0 < cnt; i0 += U * kWave) {
        Str16 kk[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          const uint32_t i = i0 + u * kWave + lane;
          kk[u] = i < cnt ? keys[s + i] : keys[s];  // key 0 again: changes neither bound
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          const uint64_t code = str27_rest_code(kk[u], false);
          lo = code < lo ? code : lo;
          hi = code > hi ? code : hi;
        }
      }
      for (int o = kWave / 2; o > 0; o >>= 1) {  // every lane holds at least one key
        const uint64_t l2 = __shfl_xor(lo, o, kWave), h2 = __shfl_xor(hi, o, kWave);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
      }
      if (lo != hi && lane == 0) {
        const uint32_t at = atomicAdd(q.list_count, 1u);
        if (at < q.list_cap) {
          q.list[at] = s;
          q.list[q.list_cap + at] = s + cnt;
        }
      }
    }

    // buckets of 2..64 keys, as many at once as fit in the 64 lanes; DEPTH
    // such lane groups are loaded before the first is ranked
    uint64_t todo = ballot(sane && cnt_l >= 2 && cnt_l <= kStrWaveBucket);
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
        k[g] = Str16{};
        v[g] = 0;
        if (valid) {
          k[g] = keys[bs[g] + (lane - boff[g])];
          if constexpr (PAIRS) v[g] = vals[bs[g] + (lane - boff[g])];
        }
      }
#pragma unroll
      for (int g = 0; g < DEPTH; ++g) {
        if (g >= ng) break;  // uniform
        const bool valid = lane < used[g];
        const uint64_t code = str27_rest_code(k[g], desc);
        // lanes of the own bucket equal so far (eq) and smaller (lt)
        uint64_t eq = active[g], lt = 0;
        for (int b = 59; b >= 0; --b) {
          const uint64_t bit = (code >> b) & 1u;
          const uint64_t B = ballot(valid && bit);
          const uint64_t spread = 0ull - bit;
          lt |= eq & ~B & spread;
          eq &= ~(B ^ spread);
          // after each symbol: stop once, within every group of lanes equal
          // so far, the bits still to come agree too (the groups can no
          // longer split, so no rank can change)
          if (b % 5 == 0 && b > 0) {
            const uint64_t rest = code & ((1ull << b) - 1);
            const int leader = valid ? __builtin_ctzll(eq) : (int)lane;
            const uint64_t lead_rest = __shfl(rest, leader, kWave);
            if (ballot(valid && rest != lead_rest) == 0) break;
          }
        }
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
