// rs_seg_kernels.h -- kernels of the batched form: many independent arrays
// (bucket sort's independent buckets, Section 2.2) sorted by one launch
// sequence whose shape depends only on the total size and the array count.
//
//   rs_seg_plan       one workgroup: splits the arrays into small ones (sorted
//                     whole on chip) and large ones, and numbers the large
//                     arrays' tiles (device side: no host round trip)
//   rs_seg_tiles      one descriptor per large-array tile
//   rs_small_sort     one workgroup per small array, every pass in LDS: count
//                     the cells, scan them, place the keys -- the hashing and
//                     extraction cycles of Sections 3.1 and 3.2 on chip
//                     (ballot ranking; 16-byte keys, one-pass plans, and
//                     arrays near the 4096-key limit)
//   rs_local_sort     the same for 4- and 8-byte keys, by 4-bit sub-passes
//                     over each cell index with per-thread counts (plans of
//                     two or more passes over short arrays, and a single
//                     short array given to rs_sort_pairs / rs_sort_keys)
//   (the large arrays' passes are rs_tile_histogram, the cell scan and
//   rs_rank_scatter<..., kPrescannedSeg>)
#pragma once

#include "rs_kernels.h"
#include "rs_seg_bounds.h"

namespace rs {

// Array s is elements [seg_lo[s], seg_hi[s]).  Offsets of back-to-back
// arrays are the case seg_hi = seg_lo + 1.
struct SegPlanParams {
  const uint64_t *seg_lo, *seg_hi;  // [nseg] each, as the caller gave them
  uint32_t nseg;
  uint32_t small_max;       // arrays up to this length are sorted on chip
  uint32_t tile;            // keys per tile of the large arrays
  uint64_t extent;          // every array lies within elements [0, extent)
  uint32_t tiles_bound;     // large-array tiles the scratch holds
  uint32_t *nlarge, *large_ids, *tile_base;  // tile_base has nlarge + 1 entries
  uint32_t *nsmall, *small_ids;
  uint64_t *rlo, *rhi;      // [nseg] each: the bounds every later kernel uses
};

// One workgroup: resolves every array's bounds, splits the arrays into
// small and large ones and numbers the large arrays' tiles array by array
// (tile_base = tiles of all earlier large arrays).
//
// The resolved bounds are the caller's, clamped so that no kernel can
// reach outside the buffers whatever the offsets hold: each array lies in
// [0, extent) and holds at most RS_MAX_ELEMENTS keys, and the large arrays
// number at most tiles_bound tiles (an array past that bound is cut to the
// tiles left, possibly none).  Valid offsets pass unchanged; invalid ones
// give an unspecified order, never an access outside keys, values or the
// scratch.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_seg_plan(const SegPlanParams q) {
  __shared__ uint32_t wsum[BLOCK / kWave];
  __shared__ uint32_t sh_large[BLOCK], sh_tiles[BLOCK], sh_small[BLOCK];
  const uint32_t t = threadIdx.x;
  uint32_t run_large = 0, run_tiles = 0, run_small = 0;
  for (uint32_t base = 0; base < q.nseg; base += BLOCK) {
    const uint32_t s = base + t;
    const bool in = s < q.nseg;
    SegBounds sb{0, 0};
    if (in) sb = resolve_segment(q.seg_lo[s], q.seg_hi[s], q.extent);
    const uint64_t lo = sb.lo;
    uint64_t len = sb.len;
    const bool large = in && len > q.small_max;
    const uint32_t want = large ? (uint32_t)((len + q.tile - 1) / q.tile) : 0u;
    sh_large[t] = large ? 1u : 0u;
    sh_tiles[t] = want;
    sh_small[t] = (in && !large) ? 1u : 0u;
    __syncthreads();
    const uint32_t tl = block_exclusive_scan<BLOCK>(sh_large, BLOCK, wsum);
    const uint32_t tt = block_exclusive_scan<BLOCK>(sh_tiles, BLOCK, wsum);
    const uint32_t ts = block_exclusive_scan<BLOCK>(sh_small, BLOCK, wsum);
    // tiles before this array, and its own, cut at the bound (run_tiles is
    // at most the bound)
    const TileRange tr = cut_tiles((uint64_t)run_tiles + sh_tiles[t], want, q.tiles_bound);
    if (large) {
      q.large_ids[run_large + sh_large[t]] = s;
      q.tile_base[run_large + sh_large[t]] = tr.first;
      const uint64_t fits = (uint64_t)(tr.last - tr.first) * q.tile;
      if (len > fits) len = fits;
    } else if (in) {
      q.small_ids[run_small + sh_small[t]] = s;
    }
    if (in) {
      q.rlo[s] = lo;
      q.rhi[s] = lo + len;
    }
    run_large += tl;
    run_tiles = cut_tiles(run_tiles, tt, q.tiles_bound).last;
    run_small += ts;
    __syncthreads();
  }
  if (t == 0) {
    *q.nlarge = run_large;
    q.tile_base[run_large] = run_tiles;
    *q.nsmall = run_small;
  }
}

struct SegTilesParams {
  const uint64_t *seg_lo, *seg_hi;
  const uint32_t *large_ids, *tile_base, *nlarge;
  uint32_t tile;
  TileDesc *tiles;   // [tiles_bound]
  uint32_t *ntotal;  // tiles in use
};

// Resolves every large-array tile id (array by array numbering) into a
// descriptor, one thread per id, so that the passes never search tables.
static __global__ __launch_bounds__(256) void rs_seg_tiles(const SegTilesParams q) {
  const uint32_t id = blockIdx.x * 256 + threadIdx.x;
  const uint32_t L = *q.nlarge;
  const uint32_t total = q.tile_base[L];
  if (id == 0) *q.ntotal = total;
  if (id >= total) return;
  uint32_t lo = 0, hi = L;  // last large array with tile_base <= id
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (q.tile_base[mid] <= id) lo = mid;
    else hi = mid;
  }
  const uint32_t sid = q.large_ids[lo];
  const uint64_t sb = q.seg_lo[sid], se = q.seg_hi[sid];
  TileDesc td;
  td.base = sb;
  td.len = (uint32_t)(se - sb);
  td.j = id - q.tile_base[lo];
  td.nt = q.tile_base[lo + 1] - q.tile_base[lo];
  td.tb = q.tile_base[lo];
  td.pad0 = td.pad1 = 0;
  q.tiles[id] = td;
}

template <class Digit>
struct SmallParams {
  Digit digit[kMaxPasses];
  uint32_t npasses;
  uint32_t pass_cells[kMaxPasses];
  const uint64_t *seg_lo, *seg_hi;
  const uint32_t *small_ids;
  const uint32_t *nsmall;
  uint64_t single_n;  // rs_local_sort without small_ids: the one array [0, single_n)
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
    const uint64_t b = sp.seg_lo[sid];
    const uint32_t len = (uint32_t)(sp.seg_hi[sid] - b);
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
      if (nvalid) {
        wave_rank<BITS, KPT>(sp.digit[pass], k, nvalid, wcnt[wave], dg, rk);
      } else {  // uniform: a wave past the end of a short array ranks nothing
#pragma unroll
        for (int r = 0; r < KPT; ++r) dg[r] = rk[r] = 0;
      }
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

// Sorts whole arrays of at most BLOCK*KPT 4- or 8-byte keys, one per
// workgroup iteration, by least-significant-first sub-passes of 4 bits over
// each pass's cell index (a stable sort by the cell index is a stable sort
// by the cell).  Thread t owns KPT consecutive positions, so the place of a
// key is: the keys of smaller sub-digit, plus the keys of equal sub-digit
// that earlier threads own, plus its rank among its own thread's equal keys.
// That is stable without comparing lanes.  Per-thread counts are 16 fields
// of 8 bits in two 64-bit registers; one LDS scan of the [sub-digit][thread]
// table turns them into starts.  LDS arrays are padded one word in 16 so
// that the blocked and striped accesses are free of bank conflicts.
template <typename K, class Digit, int BLOCK, int KPT, bool PAIRS>
__global__ __launch_bounds__(BLOCK, 4) void rs_local_sort(const SmallParams<Digit> sp, const K *__restrict__ kin,
                                                       K *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ vout) {
  static_assert(sizeof(K) <= 8 && KPT <= 16 && BLOCK % kWave == 0, "tile shape");
  constexpr uint32_t TILE = BLOCK * KPT;
  constexpr uint32_t NT = 16 * BLOCK;  // [sub-digit][thread]
  __shared__ K stage_k[TILE + TILE / 16];
  __shared__ uint32_t stage_v[PAIRS ? TILE + TILE / 16 : 1];
  __shared__ uint32_t tab[NT + NT / 16];
  __shared__ uint32_t wsum[BLOCK / kWave];
  const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const uint32_t first = t * KPT;
  const uint32_t nsmall = sp.small_ids ? *sp.nsmall : 1u;
  for (uint32_t idx = blockIdx.x; idx < nsmall; idx += gridDim.x) {
    uint64_t b = 0;
    uint32_t len = (uint32_t)sp.single_n;
    if (sp.small_ids) {
      const uint32_t sid = sp.small_ids[idx];
      b = sp.seg_lo[sid];
      len = (uint32_t)(sp.seg_hi[sid] - b);
    }
    const uint32_t nv = first >= len ? 0u : (len - first < (uint32_t)KPT ? len - first : (uint32_t)KPT);
    // coalesced loads into LDS, then each thread takes its own run
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
      const uint32_t e = r * BLOCK + t;
      if (e < len) {
        stage_k[e + (e >> 4)] = kin[b + e];
        if constexpr (PAIRS) stage_v[e + (e >> 4)] = vin[b + e];
      }
    }
    __syncthreads();
    K k[KPT];
    uint32_t v[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t i = first + j;
      if ((uint32_t)j < nv) {
        k[j] = stage_k[i + (i >> 4)];
        if constexpr (PAIRS) v[j] = stage_v[i + (i >> 4)];
      }
    }
    for (uint32_t pass = 0; pass < sp.npasses; ++pass) {
      const uint32_t cells = sp.pass_cells[pass];
      const uint32_t nbits = cells > 1 ? 32u - (uint32_t)__builtin_clz(cells - 1) : 0u;
      for (uint32_t shift = 0; shift < nbits; shift += 4) {
        // this thread's counts per sub-digit, and each key's rank among them
        uint64_t c_lo = 0, c_hi = 0;
        uint32_t rd[KPT];
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
          if ((uint32_t)j < nv) {
            const uint32_t d = (sp.digit[pass](k[j]) >> shift) & 15u;
            const uint32_t sh = (d & 7u) * 8u;
            const bool high = d >= 8;
            const uint32_t r = (uint32_t)((high ? c_hi : c_lo) >> sh) & 0xffu;
            const uint64_t inc = 1ull << sh;
            c_lo += high ? 0ull : inc;
            c_hi += high ? inc : 0ull;
            rd[j] = d << 8 | r;
          }
        }
#pragma unroll
        for (uint32_t d = 0; d < 16; ++d) {
          const uint32_t i = d * BLOCK + t;
          tab[i + (i >> 4)] = (uint32_t)((d < 8 ? c_lo : c_hi) >> ((d & 7u) * 8u)) & 0xffu;
        }
        __syncthreads();
        // exclusive scan of the table in [sub-digit][thread] order: thread
        // t owns flat entries 16t .. 16t+15 (padded: 17t .. 17t+15)
        uint32_t own[16], sum = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          own[q] = tab[17 * t + q];
          sum += own[q];
        }
        const uint32_t incl = wave_inclusive_scan(sum);
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (uint32_t w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          tab[17 * t + q] = run;
          run += own[q];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
          if ((uint32_t)j < nv) {
            const uint32_t i = (rd[j] >> 8) * BLOCK + t;
            const uint32_t pos = tab[i + (i >> 4)] + (rd[j] & 0xffu);
            stage_k[pos + (pos >> 4)] = k[j];
            if constexpr (PAIRS) stage_v[pos + (pos >> 4)] = v[j];
          }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
          const uint32_t i = first + j;
          if ((uint32_t)j < nv) {
            k[j] = stage_k[i + (i >> 4)];
            if constexpr (PAIRS) v[j] = stage_v[i + (i >> 4)];
          }
        }
      }
    }
    // stage holds the sorted array (or the input when no pass has cells)
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
      const uint32_t e = r * BLOCK + t;
      if (e < len) {
        kout[b + e] = stage_k[e + (e >> 4)];
        if constexpr (PAIRS) vout[b + e] = stage_v[e + (e >> 4)];
      }
    }
    __syncthreads();
  }
}

}  // namespace rs
