// rs_kernels.h -- gfx950 kernels of the Recombinant Sort hot path.
//
//   rs_digit_hash_histogram  the hashing cycle (Section 3.1, eq. (1)): every
//                            key's cell in every dimension group, counted in
//                            LDS tables, one read of the keys for all groups.
//   rs_tile_histogram        the same for one group, per tile of keys,
//                            written so that one flat exclusive scan of the
//                            table gives every tile's output offset per cell
//                            (for one array, or for many arrays at once).
//   rs_cell_scan             the extraction walk's running position (Section
//                            3.2): exclusive scan of cell counts in
//                            lexicographic order, single pass with decoupled
//                            look-back between chunks; rs_cell_scan_reduce /
//                            _spine / _down scan a large table in three passes;
//                            rs_group_scan scans one array's per-tile table in
//                            one launch from what rs_tile_histogram leaves.
//   rs_rank_scatter          stable emission of one dimension group: ranks
//                            each key among the tile's keys of its cell, gets
//                            the tile's offset per cell (from the scanned
//                            table, or for small arrays by look-back over the
//                            earlier tiles), and writes keys (and values)
//                            through LDS so that stores of one cell are
//                            contiguous.
//   rs_cell_count / rs_cell_emit
//                            the literal form for keys alone on a small
//                            space: count every cell of the whole space, then
//                            write each cell's count copies of the key
//                            rebuilt from its coordinates (eq. (16)).
#pragma once

#include <type_traits>

#include "rs_device.h"

namespace rs {


// ------------------------------------------------------------------ fill

// Plain copy in 4-byte words (the in-place start of an odd pass count).
static __global__ void rs_copy(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, uint64_t n4) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * 256) dst[i] = src[i];
}

static __global__ void rs_fill(uint4 *__restrict__ p, uint64_t n16, uint32_t value) {
  const uint4 v = make_uint4(value, value, value, value);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Loads VEC consecutive keys of this thread with one 128-bit load when the
// whole group is in range and the array is 16-byte aligned (`aligned`, the
// same for every thread of a launch), else one by one.
template <typename K, int VEC>
__device__ __forceinline__ void load_keys(const K *__restrict__ keys, bool aligned, uint64_t e, uint64_t end,
                                          K (&k)[VEC], bool (&valid)[VEC]) {
  if (aligned && e + VEC <= end) {
    const uint4 raw = ld_stream(reinterpret_cast<const uint4 *>(keys + e));
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
      if (valid[q]) k[q] = ld_stream(keys + e + q);
      else k[q] = K{};
    }
  }
}

// ------------------------------------------------------------- histogram

template <class Digit>
struct HistParams {
  Digit digit[kMaxPasses];  // one codec per dimension group (pass)
  uint32_t npasses;
  uint32_t stride;          // words per pass row
  uint32_t copies;          // LDS copies of the table (count_copies)
  uint64_t n;
  uint32_t *counts;         // [npasses][stride] global counts, zero before launch
  uint4 *zero;              // region cleared on the way (look-back words)
  uint64_t zero16;          // its size in 16-byte units
};

template <typename K, class Digit, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_digit_hash_histogram(const HistParams<Digit> h,
                                                                 const K *__restrict__ keys) {
  constexpr int VEC = 16 / sizeof(K);
  extern __shared__ uint32_t hist[];  // [copies][words + 1]
  const uint32_t t = threadIdx.x;
  const uint32_t words = h.npasses * h.stride, cstride = words + 1;
  for (uint32_t i = t; i < h.copies * cstride; i += BLOCK) hist[i] = 0;

  // this workgroup's share of the look-back words to clear for later passes
  {
    const uint64_t per = (h.zero16 + gridDim.x - 1) / gridDim.x;
    const uint64_t a = (uint64_t)blockIdx.x * per;
    const uint64_t b = a + per < h.zero16 ? a + per : h.zero16;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (uint64_t i = a + t; i < b; i += BLOCK) h.zero[i] = z;
  }
  __syncthreads();

  constexpr int UNROLL = 4;  // loads in flight per thread before counting
  constexpr uint64_t kStep = (uint64_t)BLOCK * VEC;
  const bool aligned = ((uintptr_t)keys % 16) == 0;
  const uint64_t per = ((h.n + gridDim.x - 1) / gridDim.x + kStep * UNROLL - 1) / (kStep * UNROLL) * (kStep * UNROLL);
  const uint64_t a = (uint64_t)blockIdx.x * per;
  const uint64_t b = a + per < h.n ? a + per : h.n;
  for (uint64_t base = a; base < b; base += kStep * UNROLL) {
    K k[UNROLL][VEC];
    bool valid[UNROLL][VEC];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
      load_keys<K, VEC>(keys, aligned, base + u * kStep + (uint64_t)t * VEC, b, k[u], valid[u]);
    for (uint32_t p = 0; p < h.npasses; ++p) {
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          lds_count(hist + p * h.stride, cstride, h.copies, valid[u][q] ? h.digit[p](k[u][q]) : 0u, valid[u][q]);
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < words; i += BLOCK) {
    uint32_t c = 0;
    for (uint32_t r = 0; r < h.copies; ++r) c += hist[r * cstride + i];
    if (c) atomicAdd(h.counts + i, c);
  }
}

// One tile of the batched form, resolved once per sort (rs_seg_tiles) so
// that the passes read it with one load instead of searching the tables.
struct alignas(16) TileDesc {
  uint64_t base;  // first key of the tile's array
  uint32_t len;   // keys in the array
  uint32_t j;     // tile index within its array
  uint32_t nt;    // tiles of the array
  uint32_t tb;    // tiles of all earlier large arrays
  uint32_t pad0, pad1;
};

// Where tile `id` lies and where its per-cell counts go in the flat table.
// One array: tile id covers keys [id * TILE, ...) and its count of cell d
// is entry d * ntiles + id.  Many arrays: entry cells * tb + d * nt + j, so
// the table holds every array's block of [cell][tile] in array order and
// one exclusive scan over it runs through arrays, then cells, then tiles:
// exactly the output order.
struct TileSpan {
  uint64_t elem0, end, base, limit;  // keys [elem0, end) of the array [base, limit)
  uint64_t entry0, estride;          // entry of cell d = entry0 + d * estride
  uint64_t block;                    // first entry of the array's block
  bool valid;
};

template <int TILE, bool SEG>
__device__ __forceinline__ TileSpan tile_span(uint64_t id, uint64_t n, uint32_t ntiles, uint32_t cells,
                                              const TileDesc *tiles, const uint32_t *ntotal) {
  TileSpan s;
  if constexpr (SEG) {
    s.valid = id < *ntotal;
    const TileDesc td = s.valid ? tiles[id] : TileDesc{0, 0, 0, 1, 0, 0, 0};
    s.base = td.base;
    s.limit = td.base + td.len;
    s.elem0 = td.base + (uint64_t)td.j * TILE;
    s.block = (uint64_t)cells * td.tb;
    s.entry0 = s.block + td.j;
    s.estride = td.nt;
  } else {
    s.valid = id < ntiles;
    s.base = 0;
    s.limit = n;
    s.elem0 = id * TILE;
    s.block = 0;
    s.entry0 = id;
    s.estride = ntiles;
  }
  s.end = s.elem0 + TILE < s.limit ? s.elem0 + TILE : s.limit;
  return s;
}

template <class Digit>
struct TileHistParams {
  Digit digit;
  uint32_t cells;    // cells of this pass's group
  uint32_t ntiles;   // one array: its tiles
  uint32_t copies;   // LDS copies per tile table
  uint64_t n;        // one array: its length
  uint32_t *counts;  // flat table (see tile_span)
  const TileDesc *tiles;   // many arrays: resolved tiles
  const uint32_t *ntotal;  // many arrays: tiles in use
  // one array (the table then feeds rs_group_scan): with several tiles per
  // workgroup the table receives each tile's count of earlier tiles of its
  // workgroup (per cell) and groups[d * ngroups + workgroup] the
  // workgroup's count of cell d (groups null: one tile per workgroup, the
  // table holds the counts); before[d * ngroups + workgroup] receives the
  // workgroup's count of all cells below d.  ngroups = the grid.
  uint32_t *groups;
  uint32_t *before;
  uint64_t ngroups;
};

// Per-tile counts of one dimension group; each workgroup takes TPW
// consecutive tiles.
template <typename K, class Digit, int BLOCK, int TPW, int TILE, bool SEG>
__global__ __launch_bounds__(BLOCK) void rs_tile_histogram(const TileHistParams<Digit> h, const K *__restrict__ keys) {
  extern __shared__ uint32_t cnt[];  // [TPW][copies][cells + 1]
  __shared__ uint64_t s_entry0[TPW], s_estride[TPW];
  const uint32_t t = threadIdx.x;
  const uint32_t cstride = h.cells + 1, tstride = h.copies * cstride;
  for (uint32_t i = t; i < TPW * tstride; i += BLOCK) cnt[i] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * TPW;
  bool whole = false;
  if constexpr (!SEG && sizeof(K) >= 16) {
    // 16-byte keys of one array, every tile of this workgroup whole and the
    // keys aligned (uniform): one flat loop of batches without bounds tests
    // (measured on 2^24 strings: 0.068 against 0.080 ms per pass; no gain
    // for 4- and 8-byte keys, which keep the loop below)
    constexpr int UNROLL = TILE / BLOCK < 4 ? TILE / BLOCK : 4;
    constexpr uint32_t BATCH = BLOCK * UNROLL;
    static_assert(TILE % BATCH == 0, "whole batches per tile");
    whole = ((uintptr_t)keys % 16) == 0 && (t0 + TPW) * TILE <= h.n;
    if (whole) {
      if (t < (uint32_t)TPW) {
        s_entry0[t] = t0 + t;
        s_estride[t] = h.ntiles;
      }
      const K *wk = keys + t0 * TILE;
      for (uint32_t b = 0; b < (uint32_t)(TPW * TILE / BATCH); ++b) {
        uint32_t *row = cnt + (b / (TILE / BATCH)) * tstride;
        K k[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) k[u] = ld_stream(wk + (uint64_t)b * BATCH + u * BLOCK + t);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) lds_count(row, cstride, h.copies, h.digit(k[u]), true);
      }
    }
  }
  for (uint32_t jj = 0; jj < (uint32_t)TPW && !whole; ++jj) {
    const TileSpan sp = tile_span<TILE, SEG>(t0 + jj, h.n, h.ntiles, h.cells, h.tiles, h.ntotal);
    if (t == 0) {
      s_entry0[jj] = sp.valid ? sp.entry0 : ~0ull;
      s_estride[jj] = sp.estride;
    }
    if (!sp.valid) continue;  // uniform
    uint32_t *row = cnt + jj * tstride;
    if constexpr (!SEG) {
      // one array: tiles start at multiples of TILE, so 128-bit loads line up
      // when the array does
      constexpr int VEC = 16 / sizeof(K);
      const bool aligned = ((uintptr_t)keys % 16) == 0;
      // four 16-byte loads in flight per thread: measured on 2^28 u32 keys
      // right after a 2 GiB write (as inside a sort), 0.173 ms against
      // 0.195 ms with eight and 0.188 ms with one
      constexpr int UNROLL = TILE / (BLOCK * VEC) < 4 ? TILE / (BLOCK * VEC) : 4;
      for (uint64_t base = sp.elem0; base < sp.end; base += (uint64_t)BLOCK * VEC * UNROLL) {
        K k[UNROLL][VEC];
        bool valid[UNROLL][VEC];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          load_keys<K, VEC>(keys, aligned, base + (uint64_t)(u * BLOCK + t) * VEC, sp.end, k[u], valid[u]);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int q = 0; q < VEC; ++q)
            lds_count(row, cstride, h.copies, valid[u][q] ? h.digit(k[u][q]) : 0u, valid[u][q]);
      }
    } else {
      constexpr int KPT = TILE / BLOCK;  // arrays start anywhere: one key per lane per load
      K k[KPT];
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const uint64_t e = sp.elem0 + (uint64_t)r * BLOCK + t;
        k[r] = e < sp.end ? keys[e] : K{};  // (non-temporal 4-byte loads measured slower here)
      }
#pragma unroll
      for (int r = 0; r < KPT; ++r) {
        const bool valid = sp.elem0 + (uint64_t)r * BLOCK + t < sp.end;
        lds_count(row, cstride, h.copies, valid ? h.digit(k[r]) : 0u, valid);
      }
    }
  }
  __syncthreads();
  if constexpr (!SEG) {
    // per cell d: the count of each tile, or with several tiles the count
    // of earlier tiles of this workgroup (into the table) and the
    // workgroup's total (into groups); a cell's TPW entries sit in TPW
    // consecutive lanes of one wave.  The workgroup's total of d replaces
    // cnt[d] (read only by the lane of tile 0 of cell d, in the same wave,
    // before), then the totals are scanned over the cells.
    static_assert(kWave % TPW == 0 && BLOCK % kWave == 0, "a cell's lanes share a wave");
    __shared__ uint32_t wsum[BLOCK / kWave];
    for (uint32_t i0 = 0; i0 < h.cells * TPW; i0 += BLOCK) {
      const uint32_t i = i0 + t;
      const bool in = i < h.cells * TPW;
      const uint32_t d = i / TPW, jj = i % TPW;
      const uint64_t e0 = in ? s_entry0[jj] : ~0ull;
      uint32_t c = 0;
      if (e0 != ~0ull)
        for (uint32_t r = 0; r < h.copies; ++r) c += cnt[jj * tstride + r * cstride + d];
      uint32_t incl = c;
#pragma unroll
      for (int o = 1; o < TPW; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, TPW);
        if (jj >= (uint32_t)o) incl += y;
      }
      if (e0 != ~0ull) h.counts[e0 + (uint64_t)d * s_estride[jj]] = TPW > 1 ? incl - c : c;
      if (in && jj == TPW - 1) {
        if constexpr (TPW > 1) h.groups[(uint64_t)d * h.ngroups + blockIdx.x] = incl;
        cnt[d] = incl;
      }
    }
    __syncthreads();
    block_exclusive_scan<BLOCK>(cnt, h.cells, wsum);
    for (uint32_t d = t; d < h.cells; d += BLOCK) h.before[(uint64_t)d * h.ngroups + blockIdx.x] = cnt[d];
    return;
  }
  // many arrays: each tile's counts
  for (uint32_t i = t; i < h.cells * TPW; i += BLOCK) {
    const uint32_t d = i / TPW, jj = i % TPW;
    const uint64_t e0 = s_entry0[jj];
    if (e0 == ~0ull) continue;
    uint32_t c = 0;
    for (uint32_t r = 0; r < h.copies; ++r) c += cnt[jj * tstride + r * cstride + d];
    h.counts[e0 + (uint64_t)d * s_estride[jj]] = c;
  }
}

// ------------------------------------------------------------- cell scan

// Traverse maps of the literal form (Section 3.1): for each value r of the
// leading coordinate (row r: cells r * inner .. r * inner + inner - 1) the
// least and greatest offset of an occupied cell in the row.  The least is
// kept complemented (nlo = ~lo, raised with atomicMax) so that one zero fill
// starts both tables: an untouched row reads lo = ~0 > hi = 0.  A
// one-dimensional space is one row.
struct RowMaps {
  uint32_t *nlo, *hi;  // [rows]
  uint32_t rows, inner;
  FastDiv32 by_inner;
};

// Largest row count of a literal space (b^2 <= 2^24 cells).
constexpr uint32_t kMaxMapRows = 4096;

// Whether some row's occupied range reaches cells [lo, hi): block-wide, the
// same answer in every thread; always true without maps (m.nlo == nullptr).
template <int BLOCK>
__device__ __forceinline__ bool chunk_occupied(const RowMaps &m, uint64_t lo, uint64_t hi) {
  if (!m.nlo) return true;
  __shared__ uint32_t s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  const uint32_t r0 = m.by_inner.div((uint32_t)lo), r1 = m.by_inner.div((uint32_t)(hi - 1));
  for (uint32_t r = r0 + threadIdx.x; r <= r1; r += BLOCK) {
    const uint32_t a = ~m.nlo[r], b = m.hi[r];
    const uint64_t first = (uint64_t)r * m.inner + a, last = (uint64_t)r * m.inner + b;
    if (a <= b && first < hi && last >= lo) s_any = 1;
  }
  __syncthreads();
  return s_any != 0;
}

struct ScanParams {
  const uint32_t *in;       // counts: [nseg][stride]
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
  for (uint32_t i = t; i < CH; i += BLOCK) vals[i] = lo + i < hi ? s.in[row + lo + i] : 0u;
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

// Three-pass exclusive scan of a large table (no chain between workgroups):
// chunk sums, a one-workgroup scan of the sums, then each chunk rescanned
// from its base.  In place (out == in) is allowed.
// The table length is `count`, or when count_dev is set *count_dev * count_mul
// (a size known only on the device); chunks past it do nothing.
__device__ __forceinline__ uint64_t scan_count(uint64_t count, const uint32_t *count_dev, uint32_t count_mul) {
  return count_dev ? (uint64_t)*count_dev * count_mul : count;
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void rs_cell_scan_reduce(const uint32_t *__restrict__ in, uint64_t count_host,
                                                             const uint32_t *count_dev, uint32_t count_mul,
                                                             uint32_t *__restrict__ sums, const RowMaps m) {
  const uint64_t count = scan_count(count_host, count_dev, count_mul);
  const uint64_t lo = (uint64_t)blockIdx.x * BLOCK * ITEMS;
  if (lo >= count) return;  // uniform
  // literal form: a chunk no occupied range reaches sums to zero unread
  const uint64_t hi_c = lo + (uint64_t)BLOCK * ITEMS < count ? lo + (uint64_t)BLOCK * ITEMS : count;
  if (!chunk_occupied<BLOCK>(m, lo, hi_c)) {
    if (threadIdx.x == 0) sums[blockIdx.x] = 0;
    return;
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint64_t e = lo + (uint64_t)i * BLOCK + threadIdx.x;
    s += e < count ? in[e] : 0u;
  }
  __shared__ uint32_t part[BLOCK / kWave];
  s = wave_sum(s);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < BLOCK / kWave; ++w) tot += part[w];
    sums[blockIdx.x] = tot;
  }
}

template <int BLOCK, int CHUNK>
__global__ __launch_bounds__(BLOCK) void rs_cell_scan_spine(uint32_t *__restrict__ sums, uint64_t count_host,
                                                            const uint32_t *count_dev, uint32_t count_mul) {
  const uint32_t nchunks = (uint32_t)((scan_count(count_host, count_dev, count_mul) + CHUNK - 1) / CHUNK);
  __shared__ uint32_t buf[BLOCK];
  __shared__ uint32_t wsum[BLOCK / kWave];
  uint32_t run = 0;
  for (uint32_t base = 0; base < nchunks; base += BLOCK) {
    const uint32_t i = base + threadIdx.x;
    buf[threadIdx.x] = i < nchunks ? sums[i] : 0u;
    __syncthreads();
    const uint32_t tot = block_exclusive_scan<BLOCK>(buf, BLOCK, wsum);
    if (i < nchunks) sums[i] = buf[threadIdx.x] + run;
    run += tot;
    __syncthreads();
  }
}

template <int BLOCK, int ITEMS, bool SPINE = false>
__global__ __launch_bounds__(BLOCK) void rs_cell_scan_down(const uint32_t *in, uint64_t count_host,
                                                           const uint32_t *count_dev, uint32_t count_mul,
                                                           const uint32_t *__restrict__ sums, uint32_t *out,
                                                           const RowMaps m) {
  constexpr uint32_t CH = BLOCK * ITEMS;
  __shared__ uint32_t vals[CH];
  __shared__ uint32_t wsum[BLOCK / kWave];
  const uint64_t count = scan_count(count_host, count_dev, count_mul);
  const uint64_t lo = (uint64_t)blockIdx.x * CH;
  if (lo >= count) return;  // uniform
  // literal form: no start is needed where nothing is emitted
  if (!chunk_occupied<BLOCK>(m, lo, lo + CH < count ? lo + CH : count)) return;
  // SPINE: the chunk sums are the reduce's, unscanned; each workgroup adds
  // up those before its chunk itself (few chunks: a small table, the
  // literal space or the string buckets), which saves the spine launch
  uint32_t spine = 0;
  if constexpr (SPINE) {
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += BLOCK) spine += sums[i];
    spine = wave_sum(spine);
    if (threadIdx.x % kWave == 0) wsum[threadIdx.x / kWave] = spine;
    __syncthreads();
    spine = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) spine += wsum[w];
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < CH; i += BLOCK) vals[i] = lo + i < count ? in[lo + i] : 0u;
  __syncthreads();
  block_exclusive_scan<BLOCK>(vals, CH, wsum);
  const uint32_t base = SPINE ? spine : sums[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < CH; i += BLOCK)
    if (lo + i < count) out[lo + i] = vals[i] + base;
}

// One array's per-tile table scanned in cell-major order in one launch:
// entry (c, t) becomes the count of every earlier cell plus the count of
// cell c in earlier tiles.  The count kernel leaves, per cell, either every
// tile's count (one tile per workgroup: the table rows are the units) or,
// with several tiles per workgroup, each tile's count of earlier tiles of
// its workgroup plus the workgroup's total in `groups` (the units); and in
// `before` each workgroup's count of the cells below c, so that a row's
// start is the sum of its `before` row: no workgroup waits for another.
// With groups, each row is split into segments of BLOCK * ITEMS tiles, one
// workgroup per segment (a segment reads only the units and its own
// entries); without, one workgroup takes the whole row (the row is scanned
// in place).
struct GroupScanParams {
  uint32_t *table;         // [cells][ntiles]
  const uint32_t *groups;  // [cells][ngroups], or null (the table rows are the units)
  const uint32_t *before;  // [cells][ngroups]
  uint64_t ntiles, ngroups;
  uint32_t shift;          // log2 of the tiles per group
  uint32_t cells, segs;    // the grid is cells * segs; segs is 1 without groups
};

template <int BLOCK>
__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t *part) {
  x = wave_sum(x);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = x;
  __syncthreads();
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / kWave; ++w) tot += part[w];
  __syncthreads();
  return tot;
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void rs_group_scan(const GroupScanParams q) {
  constexpr uint32_t CH = BLOCK * ITEMS;  // tiles per segment
  __shared__ uint32_t buf[CH];
  __shared__ uint32_t part[BLOCK / kWave];
  const uint32_t t = threadIdx.x;
  const uint32_t c = blockIdx.x / q.segs, r = blockIdx.x % q.segs;
  if (c >= q.cells) return;  // uniform
  uint32_t *row = q.table + (uint64_t)c * q.ntiles;
  const bool grouped = q.groups != nullptr;
  const uint32_t *units = grouped ? q.groups + (uint64_t)c * q.ngroups : row;
  const uint32_t *brow = q.before + (uint64_t)c * q.ngroups;
  const uint64_t t0 = (uint64_t)r * CH;
  const uint64_t tend = grouped && q.ntiles - t0 > CH ? t0 + CH : q.ntiles;
  const uint64_t u_first = t0 >> q.shift;

  // the row's start (every earlier cell) plus the units before the segment
  uint32_t s = 0;
  for (uint64_t i = t; i < q.ngroups; i += BLOCK) s += brow[i];
  for (uint64_t i = t; i < u_first; i += BLOCK) s += units[i];
  uint32_t carry = block_sum<BLOCK>(s, part);

  // BLOCK * ITEMS tiles at a time (one step with groups): their units
  // scanned in LDS
  for (uint64_t c0 = t0; c0 < tend; c0 += CH) {
    const uint32_t tn = tend - c0 < CH ? (uint32_t)(tend - c0) : CH;
    const uint64_t u0 = c0 >> q.shift;
    const uint32_t un = (uint32_t)(((c0 + tn - 1) >> q.shift) - u0 + 1);
    for (uint32_t i = t; i < un; i += BLOCK) buf[i] = units[u0 + i];
    __syncthreads();
    const uint32_t tot = block_exclusive_scan<BLOCK>(buf, un, part);
    for (uint32_t i = t; i < tn; i += BLOCK) {
      const uint64_t tile = c0 + i;
      row[tile] = carry + (grouped ? buf[(tile >> q.shift) - u0] + row[tile] : buf[i]);
    }
    carry += tot;
    __syncthreads();
  }
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

// Element i of `base` through a 32-bit byte offset (an SGPR base plus a
// 32-bit VGPR offset in the instruction) when i * sizeof(T) cannot reach
// 2^32: element types of at most 4 bytes with i below 2^30.
template <typename T>
__device__ __forceinline__ T *elem32(T *base, uint32_t i) {
  if constexpr (sizeof(T) <= 4) {
    using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T *>(reinterpret_cast<Byte *>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
  } else
    return base + i;
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

// How a tile finds its output offsets:
//   kChained       one (small) array; decoupled look-back over the earlier
//                  tiles, tile ids from an atomic counter so that every
//                  tile's predecessors are already running when it waits
//   kPrescanned    one array; offsets from the scanned per-tile table
//   kPrescannedSeg many arrays; offsets from the scanned per-tile table
enum PassMode { kChained = 0, kPrescanned = 1, kPrescannedSeg = 2 };

template <class Digit>
struct PassParams {
  Digit digit;
  uint32_t bins;                // cells of this pass's group
  uint64_t n;                   // one array: its length
  uint32_t ntiles;              // one array: its tiles
  const uint32_t *digit_start;  // kChained: exclusive scan of the pass's counts
  uint32_t *status;             // kChained: look-back words [tiles][bins], zero
  uint32_t *tile_counter;       // kChained: zero before launch
  const uint32_t *tile_offsets; // prescanned: the scanned per-tile table
  const TileDesc *tiles;        // kPrescannedSeg: resolved tiles
  const uint32_t *ntotal;       // kPrescannedSeg: tiles in use
};

// One tile = BLOCK * KPT consecutive keys.  Wave w owns keys
// [w * 64 * KPT, (w + 1) * 64 * KPT) of the tile, 64 per round, so the
// order (wave, round, lane) is the input order and every rank below is the
// number of earlier keys of the same cell: the sort is stable.
//
// Prescanned tiles do not depend on each other, so their order is chosen
// for locality: consecutive tiles run on the same XCD (workgroup b runs on
// XCD b % 8), where the partial cache lines of neighbouring tiles' output
// runs meet in one L2.  The grid is a multiple of 8; extra workgroups exit.
//
// Keys are read as KI and written as KO, and ranked as K in between: 8-byte
// keys whose space fits 32 bits are narrowed on their first pass's loads
// (KI = uint64_t, K = uint32_t) and widened on their last pass's stores.
template <typename K, class Digit, int BITS, int BLOCK, int KPT, bool PAIRS, int MODE, typename KI = K,
          typename KO = K>
__global__ __launch_bounds__(BLOCK) void rs_rank_scatter(const PassParams<Digit> p, const KI *__restrict__ kin,
                                                         KO *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                         uint32_t *__restrict__ vout) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * KPT;
  // cells of one pass: 2^BITS, except base-27 string pairs of symbols (the
  // only 16-byte passes of 10 bits), whose 729 cells need 736 table words
  // (a smaller table leaves room for one more workgroup per CU)
  constexpr int BINS = (sizeof(K) >= 16 && BITS == 10) ? 736 : (1 << BITS);
  constexpr int CPT = (BINS + BLOCK - 1) / BLOCK;  // cells per thread
  constexpr int STAGE = TILE * (sizeof(K) > 4 ? (int)sizeof(K) : 4);
  // Values get their own staging (keys and values written in one sweep)
  // when that keeps LDS within two workgroups per CU on wide tiles; else
  // they reuse the key staging after the keys are written.
  constexpr bool JOINT = PAIRS && BLOCK >= 512 &&
                         STAGE + TILE * 4 + (WAVES + 2) * BINS * 4 <= 80 * 1024;
  __shared__ __align__(16) unsigned char stage_raw[STAGE];
  __shared__ uint32_t stage_jv[JOINT ? TILE : 1];
  __shared__ uint32_t wcnt[WAVES][BINS];  // per-wave counts, then per-wave offsets
  __shared__ uint32_t tstart[BINS];       // tile-local start of each cell
  __shared__ uint32_t gdelta[BINS];       // output index - tile-local index
  __shared__ uint32_t wsum[WAVES];
  __shared__ uint64_t s_id;

  const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  K *stage_k = reinterpret_cast<K *>(stage_raw);
  uint32_t *stage_v = reinterpret_cast<uint32_t *>(stage_raw);

  for (uint32_t i = t; i < (uint32_t)(WAVES * BINS); i += BLOCK) (&wcnt[0][0])[i] = 0;
  uint64_t id;
  if constexpr (MODE == kChained) {
    if (t == 0) s_id = atomicAdd(p.tile_counter, 1u);
    __syncthreads();
    id = s_id;
  } else {
    const uint64_t per8 = gridDim.x / 8;
    id = (blockIdx.x % 8) * per8 + blockIdx.x / 8;
  }
  const TileSpan sp = tile_span<TILE, MODE == kPrescannedSeg>(id, p.n, p.ntiles, p.bins, p.tiles, p.ntotal);
  if (!sp.valid) return;  // uniform
  const uint64_t elem0 = sp.elem0, end = sp.end, out_base = sp.base, limit = sp.limit;
  const bool first_tile = id == 0;

  // ---- prescanned: this tile's output offset of each cell, relative to
  // its array, loaded together with the keys so that the tile waits for
  // memory once
  // (the array's base is subtracted only where the offsets are used, so
  // that no wait for it comes before the key loads are issued)
  uint32_t rel[CPT], rel0 = 0;
  if constexpr (MODE != kChained) {
    if constexpr (MODE == kPrescannedSeg) rel0 = p.tile_offsets[sp.block];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const uint32_t d = t + c * BLOCK;
      rel[c] = d < p.bins ? p.tile_offsets[sp.entry0 + (uint64_t)d * sp.estride] : 0u;
    }
  }

  // ---- load: keys and values of this thread, striped by rounds (offsets
  // within the tile are 32-bit)
  K k[KPT];
  uint32_t v[KPT];
  const KI *ktile = kin + elem0;
  const uint32_t *vtile = PAIRS ? vin + elem0 : nullptr;
  const uint32_t count = (uint32_t)(end - elem0);
  const uint32_t wfirst = wave * kWave * KPT + lane;
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const uint32_t e = wfirst + (uint32_t)r * kWave;
    k[r] = e < count ? (K)*elem32(ktile, e) : K{};
    if constexpr (PAIRS) v[r] = e < count ? *elem32(vtile, e) : 0u;
  }
  if constexpr (MODE != kChained) __syncthreads();  // wcnt cleared

  // ---- rank inside the wave: counts of the same cell in earlier rounds
  // (per-wave LDS counters) plus same-cell lanes below in this round.
  uint32_t dg[KPT], rk[KPT];
  const uint64_t wstart = elem0 + (uint64_t)wave * kWave * KPT;
  const uint32_t nvalid = wstart >= end ? 0u : (uint32_t)(end - wstart < (uint64_t)kWave * KPT ? end - wstart
                                                                                                : (uint64_t)kWave * KPT);
  wave_rank<BITS, KPT>(p.digit, k, nvalid, wcnt[wave], dg, rk);
  __syncthreads();

  // ---- per cell: tile count, per-wave offsets (chained: publish it)
  uint32_t tot[CPT];
  cell_totals<BLOCK, WAVES, BINS, CPT>(wcnt, tstart, p.bins, tot);
  if constexpr (MODE == kChained) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const uint32_t d = t + c * BLOCK;
      if (d < p.bins) publish(p.status + id * p.bins + d, (first_tile ? kFlagPrefix : kFlagAgg) | tot[c]);
    }
  }
  __syncthreads();
  block_exclusive_scan<BLOCK>(tstart, p.bins, wsum);

  // ---- place keys in LDS at their tile-local sorted index
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const bool valid = (uint32_t)r * kWave + lane < nvalid;
    const uint32_t lpos = tstart[dg[r]] + wcnt[wave][dg[r]] + rk[r];
    rk[r] = lpos;
    if (valid) stage_k[lpos] = k[r];
    if constexpr (JOINT)
      if (valid) stage_jv[lpos] = v[r];
  }

  // ---- each cell's output offset for this tile, relative to its array
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const uint32_t d = t + c * BLOCK;
    if (d < p.bins) {
      if constexpr (MODE == kChained) {
        uint32_t excl = 0;
        if (!first_tile) {
          excl = look_back(p.status + d, id, 0, p.bins);
          publish(p.status + id * p.bins + d, kFlagPrefix | (excl + tot[c]));
        }
        gdelta[d] = p.digit_start[d] + excl - tstart[d];
      } else {
        // wraps consistently in 32 bits: the offset relative to the array
        // is below 2^30
        gdelta[d] = rel[c] - rel0 - tstart[d];
      }
    }
  }
  __syncthreads();

  // ---- write keys (and values): consecutive LDS entries of one cell go
  // to consecutive output addresses; output offsets are relative to the
  // array and below 2^30
  KO *karr = kout + out_base;
  uint32_t *varr = PAIRS ? vout + out_base : nullptr;
  const uint32_t alen = (uint32_t)(limit - out_base);
#pragma unroll
  for (int r = 0; r < KPT; ++r) {
    const uint32_t i = t + r * BLOCK;
    if (i < count) {
      const K key = stage_k[i];
      const uint32_t d = p.digit(key);
      dg[r] = d;
      const uint32_t o = gdelta[d] + i;
      if (o < alen) {
        *elem32(karr, o) = (KO)key;
        if constexpr (JOINT) *elem32(varr, o) = stage_jv[i];
      }
    }
  }
  if constexpr (PAIRS && !JOINT) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r)
      if ((uint32_t)r * kWave + lane < nvalid) stage_v[rk[r]] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
      const uint32_t i = t + r * BLOCK;
      const uint32_t o = gdelta[dg[r]] + i;
      if (i < count && o < alen) *elem32(varr, o) = stage_v[i];
    }
  }
}

// ---------------------------------------------------- literal (keys only)

// Every key's cell of the whole space is its value (the row-major index of
// its N base-b coordinates).
template <typename K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_cell_count(const K *__restrict__ keys, uint64_t n, uint32_t cells,
                                                       uint32_t *__restrict__ counts, const RowMaps m) {
  // the hashing cycle also updates the traverse maps: this workgroup's
  // per-row least and greatest occupied offset, merged into m at the end
  extern __shared__ uint32_t maps_lds[];  // [2][rows]
  uint32_t *mnlo = maps_lds, *mhi = maps_lds + m.rows;
  for (uint32_t r = threadIdx.x; r < 2 * m.rows; r += BLOCK) maps_lds[r] = 0;
  __syncthreads();
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
    // a row's extremes settle after a few keys: read before updating
    if (valid) {
      const uint32_t r = m.by_inner.div(c), off = c - r * m.inner;
      if (~off > mnlo[r]) atomicMax(mnlo + r, ~off);
      if (off > mhi[r]) atomicMax(mhi + r, off);
    }
  }
  __syncthreads();
  // merged the same way: most workgroups find nothing to raise, and reads
  // do not queue behind one address as atomics do
  for (uint32_t r = threadIdx.x; r < m.rows; r += BLOCK)
    if (mnlo[r]) {
      if (mnlo[r] > m.nlo[r]) atomicMax(m.nlo + r, mnlo[r]);
      if (mhi[r] > m.hi[r]) atomicMax(m.hi + r, mhi[r]);
    }
}

// Writes counts[c] copies of key c at starts[c] (the extraction cycle's
// overwrite of the array).  Cells with many copies are written by the whole
// wave, 64 copies per store.
template <typename K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void rs_cell_emit(const uint32_t *__restrict__ counts,
                                                      const uint32_t *__restrict__ starts, uint32_t cells,
                                                      K *__restrict__ out, uint64_t n, const RowMaps m) {
  constexpr uint32_t kSmall = 8;
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  // the extraction walk visits only the occupied range of each row: a wave
  // whose 64 cells lie in one row, all outside its range, reads nothing
  // (every count outside the ranges is zero, so the rest need no test)
  const uint32_t cw = __builtin_amdgcn_readfirstlane(c - lane_id());
  if (cw >= cells) return;  // uniform
  const uint32_t cl = cw + kWave - 1 < cells ? cw + kWave - 1 : cells - 1;
  const uint32_t ra = m.by_inner.div(cw), rb = m.by_inner.div(cl);
  if (ra == rb) {
    const uint32_t lo = ~m.nlo[ra], hi = m.hi[ra];
    const uint32_t oa = cw - ra * m.inner, ob = cl - ra * m.inner;
    if (lo > hi || ob < lo || oa > hi) return;  // uniform
  }
  const uint32_t cnt = c < cells ? counts[c] : 0u;
  const uint32_t st = cnt ? starts[c] : 0u;
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
