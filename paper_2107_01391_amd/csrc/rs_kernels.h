// rs_kernels.h -- gfx950 kernels of the Recombinant Sort hot path.
//
//   rs_digit_hash_histogram  the hashing cycle (Section 3.1, eq. (1)): every
//                            key's cell in every dimension group, counted in
//                            LDS-private tables, one read of the keys for all
//                            groups.
//   rs_cell_scan             the extraction walk's running position (Section
//                            3.2): exclusive scan of cell counts in
//                            lexicographic order, single pass with decoupled
//                            look-back between chunks.
//   rs_rank_scatter          stable emission of one dimension group: ranks
//                            each key among the tile's keys of its cell,
//                            looks back over earlier tiles for the cell's
//                            offset, and writes keys (and values) to their
//                            final positions through LDS so that stores of
//                            one cell are contiguous.
//   rs_cell_count / rs_cell_emit
//                            the literal form for keys alone on a small
//                            space: count every cell of the whole space, then
//                            write each cell's count copies of the key
//                            rebuilt from its coordinates (eq. (16)).
#pragma once

#include "rs_device.h"

namespace rs {


// ------------------------------------------------------------------ fill

static __global__ void rs_fill(uint4 *__restrict__ p, uint64_t n16, uint32_t value) {
  const uint4 v = make_uint4(value, value, value, value);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------- histogram

template <class Digit>
struct HistParams {
  Digit digit[kMaxPasses];  // one codec per dimension group (pass)
  uint32_t npasses;
  uint32_t stride;          // words per pass row in LDS and in the partials
  uint64_t n;
  uint32_t *partials;       // [gridDim.x][npasses][stride], written whole
  uint4 *zero;              // region cleared on the way (look-back words)
  uint64_t zero16;          // its size in 16-byte units
};

// Loads VEC consecutive keys of this thread with one 128-bit load when the
// whole group is in range (keys are 16-byte aligned), else one by one.
template <typename K, int VEC>
__device__ __forceinline__ void load_keys(const K *__restrict__ keys, uint64_t e, uint64_t end, K (&k)[VEC],
                                          bool (&valid)[VEC]) {
  if (e + VEC <= end) {
    const uint4 raw = *reinterpret_cast<const uint4 *>(keys + e);
    const K *kk = reinterpret_cast<const K *>(&raw);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      k[q] = kk[q];
      valid[q] = true;
    }
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      valid[q] = e + q < end;
      if (valid[q]) k[q] = keys[e + q];
      else k[q] = K{};
    }
  }
}

template <typename K, class Digit, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_digit_hash_histogram(const HistParams<Digit> h,
                                                                 const K *__restrict__ keys) {
  constexpr int VEC = 16 / sizeof(K);
  extern __shared__ uint32_t hist[];  // [npasses][stride]
  const uint32_t t = threadIdx.x;
  const uint32_t words = h.npasses * h.stride;
  for (uint32_t i = t; i < words; i += BLOCK) hist[i] = 0;

  // this workgroup's share of the look-back words to clear for later passes
  {
    const uint64_t per = (h.zero16 + gridDim.x - 1) / gridDim.x;
    const uint64_t a = (uint64_t)blockIdx.x * per;
    const uint64_t b = a + per < h.zero16 ? a + per : h.zero16;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (uint64_t i = a + t; i < b; i += BLOCK) h.zero[i] = z;
  }
  __syncthreads();

  constexpr uint64_t kStep = (uint64_t)BLOCK * VEC;
  const uint64_t per = ((h.n + gridDim.x - 1) / gridDim.x + kStep - 1) / kStep * kStep;
  const uint64_t a = (uint64_t)blockIdx.x * per;
  const uint64_t b = a + per < h.n ? a + per : h.n;
  for (uint64_t base = a; base < b; base += kStep) {
    K k[VEC];
    bool valid[VEC];
    load_keys<K, VEC>(keys, base + (uint64_t)t * VEC, b, k, valid);
    for (uint32_t p = 0; p < h.npasses; ++p) {
      uint32_t *row = hist + p * h.stride;
#pragma unroll
      for (int q = 0; q < VEC; ++q) wave_count(row, valid[q] ? h.digit[p](k[q]) : 0u, valid[q]);
    }
  }
  __syncthreads();
  uint32_t *out = h.partials + (uint64_t)blockIdx.x * words;
  for (uint32_t i = t; i < words; i += BLOCK) out[i] = hist[i];
}

// ------------------------------------------------------------- cell scan

struct ScanParams {
  const uint32_t *in;       // counts: [nparts][nseg][stride]; summed over parts
  uint64_t part_stride;     // words between part tables
  uint32_t nparts;
  uint32_t nseg;            // independent scans
  uint32_t cells;           // cells per scan
  uint32_t stride;          // words between consecutive scans (in and out)
  uint32_t *out;            // exclusive scans [nseg][stride]
  uint32_t *chunk_status;   // [nseg * chunks_per_seg], zero before launch
  uint32_t *chunk_counter;  // zero before launch
  uint32_t chunks_per_seg;
  const uint32_t *nseg_dev;  // when set: the scans in use are *nseg_dev * nseg_mul
  uint32_t nseg_mul;
};

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void rs_cell_scan(const ScanParams s) {
  constexpr uint32_t CH = BLOCK * ITEMS;
  __shared__ uint32_t vals[CH];
  __shared__ uint32_t wsum[BLOCK / kWave];
  __shared__ uint32_t s_chunk, s_excl;
  const uint32_t t = threadIdx.x;
  if (t == 0) s_chunk = atomicAdd(s.chunk_counter, 1u);
  __syncthreads();
  const uint32_t c = s_chunk;
  if (s.nseg_dev && c >= *s.nseg_dev * s.nseg_mul * s.chunks_per_seg) return;  // uniform
  const uint32_t seg = c / s.chunks_per_seg, cc = c % s.chunks_per_seg;
  const uint32_t lo = cc * CH;
  const uint32_t hi = lo + CH < s.cells ? lo + CH : s.cells;
  const uint64_t row = (uint64_t)seg * s.stride;
  for (uint32_t i = t; i < CH; i += BLOCK) {
    uint32_t cell = lo + i, v = 0;
    if (cell < hi)
      for (uint32_t g = 0; g < s.nparts; ++g) v += s.in[g * s.part_stride + row + cell];
    vals[i] = v;
  }
  __syncthreads();
  const uint32_t total = block_exclusive_scan<BLOCK>(vals, CH, wsum);
  if (t == 0) {
    uint32_t *st = s.chunk_status + (uint64_t)seg * s.chunks_per_seg;
    uint32_t excl = 0;
    if (cc == 0) {
      publish(st, kFlagPrefix | total);
    } else {
      publish(st + cc, kFlagAgg | total);
      excl = look_back(st, cc, 0, 1);
      publish(st + cc, kFlagPrefix | (excl + total));
    }
    s_excl = excl;
  }
  __syncthreads();
  const uint32_t excl = s_excl;
  for (uint32_t i = t; lo + i < hi; i += BLOCK) s.out[row + lo + i] = vals[i] + excl;
}

// ------------------------------------------------- tile ranking helpers

// Ranks this thread's KPT keys among the keys of the same cell in its wave.
// Wave keys are taken 64 per round, so (round, lane) is input order; `my` is
// the wave's LDS counter row (zero on entry, per-cell counts on exit);
// `nvalid` is how many of the wave's 64*KPT slots hold keys.  rk[r] is the
// number of earlier keys of the wave in the same cell.
template <int BITS, int KPT, typename K, class Digit>
__device__ __forceinline__ void wave_rank(const Digit &digit, const K (&k)[KPT], uint32_t nvalid, uint32_t *my,
                                          uint32_t (&dg)[KPT], uint32_t (&rk)[KPT]) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const bool valid = (uint32_t)r * kWave + lane < nvalid;
    const uint32_t d = valid ? digit(k[r]) : 0u;
    const uint64_t peers = match_any<BITS>(d, ballot(valid));
    const uint32_t below = count_below(peers);
    uint32_t old = 0;
    if (valid) old = my[d];
    if (valid && below == 0) my[d] = old + (uint32_t)__builtin_popcountll(peers);
    dg[r] = d;
    rk[r] = old + below;
  }
}

// Per cell d handled by this thread (d = t + j*BLOCK): the tile's count,
// written to tot[j] and tstart[d], with wcnt[w][d] turned into the count of
// d in waves before w.
template <int BLOCK, int WAVES, int BINS, int CPT>
__device__ __forceinline__ void cell_totals(uint32_t (&wcnt)[WAVES][BINS], uint32_t *tstart, uint32_t bins,
                                            uint32_t (&tot)[CPT]) {
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t d = t + j * BLOCK;
    tot[j] = 0;
    if (d < bins) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = wcnt[w][d];
        wcnt[w][d] = run;
        run += c;
      }
      tot[j] = run;
      tstart[d] = run;
    }
  }
}

// ------------------------------------------------------ rank and scatter

template <class Digit>
struct PassParams {
  Digit digit;
  uint32_t bins;                // cells of this pass's group
  uint64_t n;                   // one array: its length
  const uint32_t *digit_start;  // exclusive scan of the pass's cell counts
  uint64_t dstride;             // segmented: words between segments' scans
  uint32_t *status;             // look-back words [tiles][bins], zero
  uint32_t *tile_counter;       // zero before launch
  // segmented (batched) form; unused for one array
  const uint64_t *seg_off;      // [nseg + 1]
  const uint32_t *tile_base;    // [nlarge + 1] first tile of each large array
  const uint32_t *large_ids;    // [nlarge] index of each large array
  const uint32_t *nlarge;       // device scalar
};

// One tile = BLOCK * KPT consecutive keys.  Wave w owns keys
// [w * 64 * KPT, (w + 1) * 64 * KPT) of the tile, 64 per round, so the
// order (wave, round, lane) is the input order and every rank below is the
// number of earlier keys of the same cell: the sort is stable.
template <typename K, class Digit, int BITS, int BLOCK, int KPT, bool PAIRS, bool SEG>
__global__ __launch_bounds__(BLOCK) void rs_rank_scatter(const PassParams<Digit> p, const K *__restrict__ kin,
                                                         K *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                         uint32_t *__restrict__ vout) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * KPT;
  constexpr int BINS = 1 << BITS;
  constexpr int CPT = (BINS + BLOCK - 1) / BLOCK;  // cells per thread
  constexpr int STAGE = TILE * (sizeof(K) > 4 ? (int)sizeof(K) : 4);
  __shared__ __align__(16) unsigned char stage_raw[STAGE];
  __shared__ uint32_t wcnt[WAVES][BINS];  // per-wave counts, then per-wave offsets
  __shared__ uint32_t tstart[BINS];       // tile-local start of each cell
  __shared__ uint32_t gdelta[BINS];       // output index - tile-local index
  __shared__ uint32_t wsum[WAVES];
  __shared__ uint64_t s_tile, s_first, s_elem0, s_end, s_seg, s_row;

  const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  K *stage_k = reinterpret_cast<K *>(stage_raw);
  uint32_t *stage_v = reinterpret_cast<uint32_t *>(stage_raw);

  for (uint32_t i = t; i < (uint32_t)(WAVES * BINS); i += BLOCK) (&wcnt[0][0])[i] = 0;
  if (t == 0) {
    const uint64_t tile = atomicAdd(p.tile_counter, 1u);
    if constexpr (!SEG) {
      s_tile = tile;
      s_first = 0;
      s_elem0 = tile * TILE;
      s_end = s_elem0 + TILE < p.n ? s_elem0 + TILE : p.n;
      s_seg = 0;
      s_row = 0;
    } else {
      const uint32_t L = *p.nlarge;
      if (tile >= p.tile_base[L]) {
        s_tile = ~0ull;
      } else {
        uint32_t lo = 0, hi = L;  // last j with tile_base[j] <= tile
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) / 2;
          if (p.tile_base[mid] <= tile) lo = mid;
          else hi = mid;
        }
        const uint32_t sid = p.large_ids[lo];
        const uint64_t sb = p.seg_off[sid], se = p.seg_off[sid + 1];
        s_tile = tile;
        s_first = p.tile_base[lo];
        s_elem0 = sb + (tile - s_first) * TILE;
        s_end = s_elem0 + TILE < se ? s_elem0 + TILE : se;
        s_seg = sid;
        s_row = lo;
      }
    }
  }
  __syncthreads();
  const uint64_t tile = s_tile;
  if (SEG && tile == ~0ull) return;
  const uint64_t first = s_first, elem0 = s_elem0, end = s_end;
  const uint64_t out_base = SEG ? p.seg_off[s_seg] : 0;
  const uint64_t limit = SEG ? p.seg_off[s_seg + 1] : p.n;  // no store leaves the array
  const uint32_t *dstart = SEG ? p.digit_start + s_row * p.dstride : p.digit_start;

  // ---- load: keys and values of this thread, striped by rounds
  K k[KPT];
  uint32_t v[KPT];
  const uint64_t wbase = elem0 + (uint64_t)wave * kWave * KPT + lane;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const uint64_t e = wbase + (uint64_t)r * kWave;
    k[r] = e < end ? kin[e] : K{};
    if constexpr (PAIRS) v[r] = e < end ? vin[e] : 0u;
  }

  // ---- rank inside the wave: counts of the same cell in earlier rounds
  // (per-wave LDS counters) plus same-cell lanes below in this round.
  uint32_t dg[KPT], rk[KPT];
  const uint64_t wstart = elem0 + (uint64_t)wave * kWave * KPT;
  const uint32_t nvalid = wstart >= end ? 0u : (uint32_t)(end - wstart < (uint64_t)kWave * KPT ? end - wstart
                                                                                                : (uint64_t)kWave * KPT);
  wave_rank<BITS, KPT>(p.digit, k, nvalid, wcnt[wave], dg, rk);
  __syncthreads();

  // ---- per cell: tile count, per-wave offsets, publish the tile's count
  uint32_t tot[CPT];
  cell_totals<BLOCK, WAVES, BINS, CPT>(wcnt, tstart, p.bins, tot);
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t d = t + j * BLOCK;
    if (d < p.bins) publish(p.status + tile * p.bins + d, (tile == first ? kFlagPrefix : kFlagAgg) | tot[j]);
  }
  __syncthreads();
  block_exclusive_scan<BLOCK>(tstart, p.bins, wsum);

  // ---- look back over earlier tiles of this array for each cell's offset
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t d = t + j * BLOCK;
    if (d < p.bins) {
      uint32_t excl = 0;
      if (tile != first) {
        excl = look_back(p.status + d, tile, first, p.bins);
        publish(p.status + tile * p.bins + d, kFlagPrefix | (excl + tot[j]));
      }
      gdelta[d] = dstart[d] + excl - tstart[d];
    }
  }

  // ---- place keys in LDS at their tile-local sorted index
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const bool valid = wbase + (uint64_t)r * kWave < end;
    const uint32_t lpos = tstart[dg[r]] + wcnt[wave][dg[r]] + rk[r];
    rk[r] = lpos;
    if (valid) stage_k[lpos] = k[r];
  }
  __syncthreads();

  // ---- write keys: consecutive LDS entries of one cell go to consecutive
  // output addresses
  const uint32_t count = (uint32_t)(end - elem0);
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t i = t + j * BLOCK;
    if (i < count) {
      const K key = stage_k[i];
      const uint32_t d = p.digit(key);
      dg[j] = d;
      const uint64_t at = out_base + gdelta[d] + i;
      if (at < limit) kout[at] = key;
    }
  }
  if constexpr (PAIRS) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r)
      if (wbase + (uint64_t)r * kWave < end) stage_v[rk[r]] = v[r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const uint32_t i = t + j * BLOCK;
      const uint64_t at = out_base + gdelta[dg[j]] + i;
      if (i < count && at < limit) vout[at] = stage_v[i];
    }
  }
}

// ---------------------------------------------------- literal (keys only)

// Every key's cell of the whole space is its value (the row-major index of
// its N base-b coordinates).
template <typename K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_cell_count(const K *__restrict__ keys, uint64_t n, uint32_t cells,
                                                       uint32_t *__restrict__ counts) {
  for (uint64_t e = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; e - threadIdx.x < n;
       e += (uint64_t)gridDim.x * BLOCK) {
    const bool valid = e < n;
    // a key outside the space (invalid input) is clamped to its last cell
    const uint64_t key = valid ? (uint64_t)keys[e] : 0u;
    const uint32_t c = key < cells ? (uint32_t)key : cells - 1;
    const uint64_t act = ballot(valid);
    const uint32_t first = (uint32_t)__builtin_ctzll(act);
    const uint32_t c0 = __builtin_amdgcn_readlane(c, first);
    if (ballot(valid && c == c0) == act) {
      if (lane_id() == first) atomicAdd(counts + c0, (uint32_t)__builtin_popcountll(act));
    } else if (valid) {
      atomicAdd(counts + c, 1u);
    }
  }
}

// Writes counts[c] copies of key c at starts[c] (the extraction cycle's
// overwrite of the array).  Cells with many copies are written by the whole
// wave, 64 copies per store.
template <typename K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_cell_emit(const uint32_t *__restrict__ counts,
                                                      const uint32_t *__restrict__ starts, uint32_t cells,
                                                      K *__restrict__ out, uint64_t n) {
  constexpr uint32_t kSmall = 8;
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t cnt = c < cells ? counts[c] : 0u;
  const uint32_t st = c < cells ? starts[c] : 0u;
  if (cnt <= kSmall) {
    for (uint32_t z = 0; z < cnt; ++z)
      if (st + z < n) out[st + z] = (K)c;
  }
  uint64_t big = ballot(cnt > kSmall);
  const uint32_t lane = lane_id();
  while (big) {
    const uint32_t l = (uint32_t)__builtin_ctzll(big);
    big &= big - 1;
    const uint32_t cl = __builtin_amdgcn_readlane(c, l);
    const uint32_t nl = __builtin_amdgcn_readlane(cnt, l);
    const uint32_t sl = __builtin_amdgcn_readlane(st, l);
    for (uint32_t z = lane; z < nl; z += kWave)
      if (sl + z < n) out[sl + z] = (K)cl;
  }
}

}  // namespace rs
