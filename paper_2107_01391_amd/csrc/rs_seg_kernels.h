// rs_seg_kernels.h -- kernels of the batched form: many independent arrays
// (bucket sort's independent buckets, Section 2.2) sorted by one launch
// sequence whose shape depends only on the total size and the array count.
//
//   rs_seg_plan       one workgroup: splits the arrays into small ones (sorted
//                     whole on chip) and large ones, and numbers the large
//                     arrays' tiles (device side: no host round trip)
//   rs_small_sort     one workgroup per small array, every pass in LDS: count
//                     the cells, scan them, place the keys -- the hashing and
//                     extraction cycles of Sections 3.1 and 3.2 on chip
//   rs_seg_histogram  per large array, every pass's cell counts in one read
//   (the passes themselves are rs_rank_scatter<..., SEG = true>)
#pragma once

#include "rs_kernels.h"

namespace rs {

struct SegPlanParams {
  const uint64_t *seg_off;  // [nseg + 1]
  uint32_t nseg;
  uint32_t small_max;       // arrays up to this length are sorted on chip
  uint32_t tile;            // keys per tile of the large arrays
  uint32_t *nlarge, *large_ids, *tile_base;  // tile_base has nlarge + 1 entries
  uint32_t *nsmall, *small_ids;
};

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_seg_plan(const SegPlanParams q) {
  __shared__ uint32_t wsum[BLOCK / kWave];
  __shared__ uint32_t sh_large[BLOCK], sh_tiles[BLOCK], sh_small[BLOCK];
  const uint32_t t = threadIdx.x;
  uint32_t run_large = 0, run_tiles = 0, run_small = 0;
  for (uint32_t base = 0; base < q.nseg; base += BLOCK) {
    const uint32_t s = base + t;
    uint64_t len = 0;
    if (s < q.nseg) len = q.seg_off[s + 1] - q.seg_off[s];
    const bool in = s < q.nseg;
    const bool large = in && len > q.small_max;
    sh_large[t] = large ? 1u : 0u;
    sh_tiles[t] = large ? (uint32_t)((len + q.tile - 1) / q.tile) : 0u;
    sh_small[t] = (in && !large) ? 1u : 0u;
    __syncthreads();
    const uint32_t tl = block_exclusive_scan<BLOCK>(sh_large, BLOCK, wsum);
    const uint32_t tt = block_exclusive_scan<BLOCK>(sh_tiles, BLOCK, wsum);
    const uint32_t ts = block_exclusive_scan<BLOCK>(sh_small, BLOCK, wsum);
    if (large) {
      q.large_ids[run_large + sh_large[t]] = s;
      q.tile_base[run_large + sh_large[t]] = run_tiles + sh_tiles[t];
    } else if (in) {
      q.small_ids[run_small + sh_small[t]] = s;
    }
    run_large += tl;
    run_tiles += tt;
    run_small += ts;
    __syncthreads();
  }
  if (t == 0) {
    *q.nlarge = run_large;
    q.tile_base[run_large] = run_tiles;
    *q.nsmall = run_small;
  }
}

template <class Digit>
struct SmallParams {
  Digit digit[kMaxPasses];
  uint32_t npasses;
  uint32_t pass_cells[kMaxPasses];
  const uint64_t *seg_off;
  const uint32_t *small_ids;
  const uint32_t *nsmall;
};

// Sorts whole arrays of at most BLOCK*KPT keys, one per workgroup iteration.
// Keys stay in registers between passes; each pass ranks them per wave,
// scans the tile's cell counts and places keys (and values) in LDS at their
// new index, then reads them back in the same striped order.
template <typename K, class Digit, int BITS, int BLOCK, int KPT, bool PAIRS>
__global__ __launch_bounds__(BLOCK) void rs_small_sort(const SmallParams<Digit> sp, const K *__restrict__ kin,
                                                       K *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ vout) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * KPT;
  constexpr int BINS = 1 << BITS;
  constexpr int CPT = (BINS + BLOCK - 1) / BLOCK;
  __shared__ __align__(16) K stage_k[TILE];
  __shared__ uint32_t stage_v[PAIRS ? TILE : 1];
  __shared__ uint32_t wcnt[WAVES][BINS];
  __shared__ uint32_t tstart[BINS];
  __shared__ uint32_t wsum[WAVES];
  const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const uint32_t nsmall = *sp.nsmall;
  for (uint32_t idx = blockIdx.x; idx < nsmall; idx += gridDim.x) {
    const uint32_t sid = sp.small_ids[idx];
    const uint64_t b = sp.seg_off[sid];
    const uint32_t len = (uint32_t)(sp.seg_off[sid + 1] - b);
    const uint32_t wstart = wave * kWave * KPT;
    const uint32_t nvalid = wstart >= len ? 0u : (len - wstart < (uint32_t)(kWave * KPT) ? len - wstart
                                                                                          : (uint32_t)(kWave * KPT));
    K k[KPT];
    uint32_t v[KPT];
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
      const uint32_t e = wstart + r * kWave + lane;
      k[r] = e < len ? kin[b + e] : K{};
      if constexpr (PAIRS) v[r] = e < len ? vin[b + e] : 0u;
    }
    for (uint32_t pass = 0; pass < sp.npasses; ++pass) {
      const uint32_t cells = sp.pass_cells[pass];
      for (uint32_t i = t; i < (uint32_t)(WAVES * BINS); i += BLOCK) (&wcnt[0][0])[i] = 0;
      __syncthreads();
      uint32_t dg[KPT], rk[KPT];
      wave_rank<BITS, KPT>(sp.digit[pass], k, nvalid, wcnt[wave], dg, rk);
      __syncthreads();
      uint32_t tot[CPT];
      cell_totals<BLOCK, WAVES, BINS, CPT>(wcnt, tstart, cells, tot);
      __syncthreads();
      block_exclusive_scan<BLOCK>(tstart, cells, wsum);
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        if ((uint32_t)r * kWave + lane < nvalid) {
          const uint32_t lpos = tstart[dg[r]] + wcnt[wave][dg[r]] + rk[r];
          stage_k[lpos] = k[r];
          if constexpr (PAIRS) stage_v[lpos] = v[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const uint32_t e = wstart + r * kWave + lane;
        if (e < len) {
          k[r] = stage_k[e];
          if constexpr (PAIRS) v[r] = stage_v[e];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
      const uint32_t e = wstart + r * kWave + lane;
      if (e < len) {
        kout[b + e] = k[r];
        if constexpr (PAIRS) vout[b + e] = v[r];
      }
    }
  }
}

template <class Digit>
struct SegHistParams {
  Digit digit[kMaxPasses];
  uint32_t npasses;
  uint32_t stride;            // words per (array, pass) row
  uint32_t tile;              // keys per tile
  const uint64_t *seg_off;
  const uint32_t *tile_base;  // [nlarge + 1]
  const uint32_t *large_ids;
  const uint32_t *nlarge;
  uint32_t *seg_hist;         // [nlarge][npasses][stride], zero before launch
  uint4 *zero;                // look-back words to clear
  uint64_t zero16;
};

// Each workgroup takes a contiguous run of tiles; counts accumulate in LDS
// while the run stays in one array and are added to that array's global
// table when it changes, so an array costs one flush per workgroup touching
// it rather than one per tile.
template <typename K, class Digit, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_seg_histogram(const SegHistParams<Digit> h, const K *__restrict__ keys) {
  extern __shared__ uint32_t hist[];  // [npasses][stride]
  __shared__ uint32_t s_row;
  const uint32_t t = threadIdx.x;
  const uint32_t words = h.npasses * h.stride;
  {
    const uint64_t per = (h.zero16 + gridDim.x - 1) / gridDim.x;
    const uint64_t a = (uint64_t)blockIdx.x * per;
    const uint64_t b = a + per < h.zero16 ? a + per : h.zero16;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (uint64_t i = a + t; i < b; i += BLOCK) h.zero[i] = z;
  }
  const uint32_t L = *h.nlarge;
  const uint32_t T = h.tile_base[L];
  const uint32_t per = (T + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = t0 + per < T ? t0 + per : T;
  if (t0 >= t1) return;
  for (uint32_t i = t; i < words; i += BLOCK) hist[i] = 0;
  if (t == 0) {
    uint32_t lo = 0, hi = L;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) / 2;
      if (h.tile_base[mid] <= t0) lo = mid;
      else hi = mid;
    }
    s_row = lo;
  }
  __syncthreads();
  uint32_t row = s_row;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    while (tile >= h.tile_base[row + 1]) ++row;  // uniform: every thread walks the same rows
    const uint32_t sid = h.large_ids[row];
    const uint64_t sb = h.seg_off[sid], se = h.seg_off[sid + 1];
    const uint64_t e0 = sb + (uint64_t)(tile - h.tile_base[row]) * h.tile;
    const uint64_t e1 = e0 + h.tile < se ? e0 + h.tile : se;
    for (uint64_t base = e0; base < e1; base += BLOCK) {
      const uint64_t e = base + t;
      const bool valid = e < e1;
      const K key = valid ? keys[e] : K{};
      for (uint32_t p = 0; p < h.npasses; ++p) wave_count(hist + p * h.stride, valid ? h.digit[p](key) : 0u, valid);
    }
    const bool last_of_row = (tile + 1 == t1) || (tile + 1 >= h.tile_base[row + 1]);
    if (last_of_row) {
      __syncthreads();
      uint32_t *dst = h.seg_hist + (uint64_t)row * words;
      for (uint32_t i = t; i < words; i += BLOCK) {
        const uint32_t c = hist[i];
        if (c) atomicAdd(dst + i, c);
        hist[i] = 0;
      }
      __syncthreads();
    }
  }
}

}  // namespace rs
