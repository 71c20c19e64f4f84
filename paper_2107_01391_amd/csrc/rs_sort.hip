// rs_sort.hip -- C ABI and launch sequences of the single-array sort.
//
// rs_sort_pairs / rs_sort_keys, chained passes (small arrays):
//   1. rs_fill                 clear the control words and count tables
//   2. rs_digit_hash_histogram one read of the keys: every pass's cell counts,
//                              clears the look-back words on the way
//   3. rs_cell_scan            exclusive scan of every pass's counts
//   4. rs_rank_scatter x P     stable passes, least significant group first,
//                              ping-ponging between the output and scratch
// prescanned passes (large arrays), per pass (rs_passes.h):
//   1. rs_tile_histogram       per-tile counts of the pass's group
//   2. rs_group_scan           one exclusive scan of that table (one launch;
//                              many arrays: rs_cell_scan_reduce/_spine/_down),
//                              cell-major: every tile's output offset per cell
//   3. rs_rank_scatter         stable scatter, offsets read from the table
// rs_sort_keys on a small space (literal):
//   1. rs_fill                 clear the cell counts
//   2. rs_cell_count           S[cell]++ over the whole space
//   3. rs_cell_scan            running output position per cell
//   4. rs_cell_emit            count copies of each cell's rebuilt key
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "rs_internal.h"
#include "rs_kernels.h"
#include "rs_passes.h"
#include "rs_seg_kernels.h"
#include "rs_segmented.h"
#include "rs_str_buckets.h"

namespace rs {

thread_local std::string g_last_error;

rs_status fail(rs_status st, const std::string &why) {
  g_last_error = why;
  return st;
}

int cu_count() {
  static int cached = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cached = cus;
    if (cached <= 0) cached = 256;
  });
  return cached;
}

rs_status check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return RS_OK;
}

rs_status launch_fill(void *p, size_t bytes, uint32_t value, hipStream_t stream) {
  if (bytes == 0) return RS_OK;
  const uint64_t n16 = bytes / 16;
  uint64_t blocks = (n16 + 255) / 256;
  const uint64_t cap = (uint64_t)cu_count() * 8;
  if (blocks > cap) blocks = cap;
  if (blocks == 0) blocks = 1;
  RS_TIMED("rs_fill", stream, hipLaunchKernelGGL(rs_fill, dim3((uint32_t)blocks), dim3(256), 0, stream, (uint4 *)p, n16, value));
  return check_launch("rs_fill");
}

rs_status launch_copy(void *dst, const void *src, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return RS_OK;
  const uint64_t n4 = bytes / 4;
  uint64_t blocks = (n4 + 255) / 256;
  const uint64_t cap = (uint64_t)cu_count() * 8;
  if (blocks > cap) blocks = cap;
  RS_TIMED("rs_copy", stream,
           hipLaunchKernelGGL(rs_copy, dim3((uint32_t)blocks), dim3(256), 0, stream, (uint32_t *)dst,
                              (const uint32_t *)src, n4));
  return check_launch("rs_copy");
}

// --------------------------------------------------------- grouped passes

template <typename K, class Digit, int BITS>
static rs_status run_passes(const Plan &pl, const Digit *digits, const void *keys_in, void *keys_out,
                            const uint32_t *vals_in, uint32_t *vals_out, void *tmp, hipStream_t stream) {
  char *base = (char *)tmp;
  uint32_t *ctrl = (uint32_t *)(base + pl.off_ctrl);
  uint32_t *counts = ctrl + pl.npasses + 1 + pl.scan_chunks;  // [P][bins]
  uint32_t *dstart = (uint32_t *)(base + pl.off_dstart);
  uint32_t *status = (uint32_t *)(base + pl.off_status);
  rs_status st = launch_fill(ctrl, pl.ctrl_bytes, 0, stream);
  if (st != RS_OK) return st;

  // 2. histogram of every pass in one read
  HistParams<Digit> h;
  memset(&h, 0, sizeof h);
  for (uint32_t i = 0; i < pl.npasses; ++i) h.digit[i] = digits[i];
  h.npasses = pl.npasses;
  h.stride = pl.bins;
  h.copies = pl.hist_copies;
  h.n = pl.n;
  h.counts = counts;
  h.zero = (uint4 *)status;
  h.zero16 = pl.status_bytes / 16;
  const size_t lds = (size_t)pl.hist_copies * (pl.npasses * pl.bins + 1) * 4;
  RS_TIMED("rs_digit_hash_histogram", stream,
           hipLaunchKernelGGL((rs_digit_hash_histogram<K, Digit, 256>), dim3(pl.hist_grid), dim3(256), lds, stream,
                              h, (const K *)keys_in));
  if ((st = check_launch("rs_digit_hash_histogram")) != RS_OK) return st;

  // 3. exclusive scan of each pass's cells
  ScanParams s;
  memset(&s, 0, sizeof s);  // no traverse maps unless set
  s.in = counts;
  s.nseg = pl.npasses;
  s.cells = pl.bins;
  s.stride = pl.bins;
  s.out = dstart;
  s.chunk_counter = ctrl + pl.npasses;
  s.chunk_status = ctrl + pl.npasses + 1;
  s.chunks_per_seg = (pl.bins + kScanChunk - 1) / kScanChunk;
  s.nseg_dev = nullptr;
  s.nseg_mul = 1;
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan<kScanBlock, kScanItems>), dim3(s.nseg * s.chunks_per_seg),
                              dim3(kScanBlock), 0, stream, s));
  if ((st = check_launch("rs_cell_scan")) != RS_OK) return st;

  // 4. stable passes; buffer X = output, Y = scratch; pass P-1 writes X
  const size_t kb = pl.key.key_bytes;
  K *X = (K *)keys_out;
  K *Y = (K *)(base + pl.off_keys_alt);
  uint32_t *XV = vals_out;
  uint32_t *YV = (uint32_t *)(base + pl.off_vals_alt);
  const K *src = (const K *)keys_in;
  const uint32_t *srcv = vals_in;
  const bool odd = pl.npasses % 2 == 1;
  if (odd && keys_in == keys_out) {
    // pass 0 would read and write X: start from a copy in Y
    if ((st = launch_copy(Y, keys_in, pl.n * kb, stream)) != RS_OK) return st;
    src = Y;
  }
  if (pl.pairs && odd && vals_in == vals_out) {
    if ((st = launch_copy(YV, vals_in, pl.n * 4, stream)) != RS_OK) return st;
    srcv = YV;
  }
  for (uint32_t i = 0; i < pl.npasses; ++i) {
    const bool to_x = ((pl.npasses - 1 - i) % 2) == 0;
    K *dst = to_x ? X : Y;
    uint32_t *dstv = to_x ? XV : YV;
    PassParams<Digit> pp;
    memset(&pp, 0, sizeof pp);
    pp.digit = digits[i];
    pp.bins = pl.pass_cells[i];
    pp.n = pl.n;
    pp.digit_start = dstart + (size_t)i * pl.bins;
    pp.status = status + (size_t)i * pl.ntiles * pl.bins;
    pp.tile_counter = ctrl + i;
    pp.ntiles = (uint32_t)pl.ntiles;
    const dim3 blk(256);
    constexpr int KPT = sizeof(K) >= 16 ? 8 : 16;  // LDS staging of one tile: 32 KiB at most
    if (pl.pairs) {
      auto kern = rs_rank_scatter<K, Digit, BITS, 256, KPT, true, kChained>;
      const dim3 grid((uint32_t)pl.ntiles);
      RS_TIMED("rs_rank_scatter", stream, hipLaunchKernelGGL(kern, grid, blk, 0, stream, pp, src, dst, srcv, dstv));
    } else {
      auto kern = rs_rank_scatter<K, Digit, BITS, 256, KPT, false, kChained>;
      const dim3 grid((uint32_t)pl.ntiles);
      RS_TIMED("rs_rank_scatter", stream,
               hipLaunchKernelGGL(kern, grid, blk, 0, stream, pp, src, dst, nullptr, nullptr));
    }
    if ((st = check_launch("rs_rank_scatter")) != RS_OK) return st;
    src = dst;
    srcv = dstv;
  }
  return RS_OK;
}

// Workgroups of 256 threads of a kernel that run at once on the whole chip.
template <auto KERNEL>
static uint32_t resident_grid() {
  static uint32_t grid = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, KERNEL, 256, 0) != hipSuccess || per_cu <= 0) {
      (void)hipGetLastError();  // the query's error is not a launch's
      per_cu = 4;
    }
    grid = (uint32_t)per_cu * (uint32_t)cu_count();
  });
  return grid;
}

// Base-27 strings of 16 symbols by buckets (rs_str_buckets.h): the two
// passes over the four leading symbols order the array by its 27^4 leading
// cells; each cell's bucket is then sorted by the twelve other symbols, in
// place in the output.  Buckets of more than 64 keys that are not all equal
// in those symbols, if any, are listed on the device; the list's length is
// read back (the one synchronisation of this form) and they go through the
// batched passes over the twelve symbols.
static rs_status run_str_buckets(const Plan &pl, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                                 uint32_t *vals_out, void *tmp, hipStream_t stream) {
  char *base = (char *)tmp;
  const bool pairs = pl.pairs;
  Str16 *X = (Str16 *)keys_out;
  Str16 *Y = (Str16 *)(base + pl.off_keys_alt);
  uint32_t *YV = pairs ? (uint32_t *)(base + pl.off_vals_alt) : nullptr;
  uint32_t *table = (uint32_t *)(base + pl.off_table), *sums = (uint32_t *)(base + pl.off_sums);
  // passes 6 (symbols 2, 3) and 7 (symbols 0, 1) of the least-significant-
  // first order: keys_in -> Y -> X
  rs_status st = prescanned_pass<Str16, DigitStr16, 10, 256, false>(
      pl.s16[6], pl.pass_cells[6], pairs, (const Str16 *)keys_in, Y, vals_in, YV, pl.n, pl.ntiles, table, sums,
      nullptr, nullptr, stream);
  if (st != RS_OK) return st;
  st = prescanned_pass<Str16, DigitStr16, 10, 256, false>(pl.s16[7], pl.pass_cells[7], pairs, Y, X, YV, vals_out,
                                                          pl.n, pl.ntiles, table, sums, nullptr, nullptr, stream);
  if (st != RS_OK) return st;

  // S of the four leading symbols, and each bucket's start
  StrBucketParams q;
  memset(&q, 0, sizeof q);
  q.lead_cx = pl.key.descending ? ~0u : 0u;
  q.lead_ca = pl.key.descending ? kStrBucketCells : 0u;
  q.n = pl.n;
  q.counts = (uint32_t *)(base + pl.off_bcounts);
  q.mixed = (uint8_t *)(base + pl.off_bmixed);
  q.starts = (uint32_t *)(base + pl.off_bstarts);
  q.list = (uint64_t *)(base + pl.off_blist);
  q.list_count = (uint32_t *)(base + pl.off_bctrl);
  q.list_cap = pl.blist_cap;
  q.descending = pl.key.descending ? 1u : 0u;
  if ((st = launch_fill(q.counts, pl.bfill_bytes, 0, stream)) != RS_OK) return st;
  // one contiguous range of the array per wave, as many waves as the chip
  // holds at once
  RS_TIMED("rs_str_bucket_count", stream,
           hipLaunchKernelGGL((rs_str_bucket_count<256>), dim3(resident_grid<rs_str_bucket_count<256>>()), dim3(256),
                              0, stream, q, X));
  if ((st = check_launch("rs_str_bucket_count")) != RS_OK) return st;
  const uint64_t cells = kStrBucketCells;
  const uint32_t nchunks = (uint32_t)((cells + kBigScanChunk - 1) / kBigScanChunk);
  uint32_t *bsums = (uint32_t *)(base + pl.off_bsums);
  RowMaps nomaps;
  memset(&nomaps, 0, sizeof nomaps);
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan_reduce<kScanBlock, kBigScanItems>), dim3(nchunks), dim3(kScanBlock), 0,
                              stream, q.counts, cells, nullptr, 1, bsums, nomaps));
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan_down<kScanBlock, kBigScanItems, true>), dim3(nchunks), dim3(kScanBlock), 0,
                              stream, q.counts, cells, nullptr, 1, bsums, (uint32_t *)q.starts, nomaps));
  if ((st = check_launch("rs_cell_scan")) != RS_OK) return st;

  // the mixed buckets: as many waves as the chip holds at once, each over
  // an equal run of cells
  if (pairs)
    RS_TIMED("rs_str_bucket_sort", stream,
             hipLaunchKernelGGL((rs_str_bucket_sort<256, true>), dim3(resident_grid<rs_str_bucket_sort<256, true>>()), dim3(256), 0, stream,
                                q, X, vals_out));
  else
    RS_TIMED("rs_str_bucket_sort", stream,
             hipLaunchKernelGGL((rs_str_bucket_sort<256, false>), dim3(resident_grid<rs_str_bucket_sort<256, false>>()), dim3(256), 0,
                                stream, q, X, nullptr));
  if ((st = check_launch("rs_str_bucket_sort")) != RS_OK) return st;

  uint32_t nlong = 0;
  if (hipMemcpyAsync(&nlong, q.list_count, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(RS_ERR_HIP, "reading the count of long buckets");
  if (nlong == 0) return RS_OK;
  if (nlong > pl.blist_cap) return fail(RS_ERR_HIP, "long-bucket list overflow");
  // the listed long buckets: the batched passes over the twelve
  // symbols, in place, with the alternate arrays as their scratch
  SegLayout L;
  std::string why;
  if ((st = make_seg_layout(pl, 6, pl.n, pl.n, nlong, false, 256, &L, &why)) != RS_OK) return fail(st, why);
  if (L.bytes > pl.bseg.bytes) return fail(RS_ERR_HIP, "long-bucket layout exceeds its scratch");
  return run_segmented<Str16, DigitStr16, 10>(pl, L, pl.s16, X, X, pairs ? vals_out : nullptr,
                                              pairs ? vals_out : nullptr, Y, YV, q.list, q.list + pl.blist_cap,
                                              base + pl.off_bseg, stream);
}

template <typename K, class Digit, int BITS>
static rs_status run_prescanned(const Plan &pl, const Digit *digits, const void *keys_in, void *keys_out,
                                const uint32_t *vals_in, uint32_t *vals_out, void *tmp, hipStream_t stream) {
  char *base = (char *)tmp;
  if constexpr (std::is_same<K, Str16>::value && BITS == 10) {
    if (pl.str_buckets) {
      hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
      // a captured sequence cannot wait for the long-bucket count: all
      // eight passes then
      if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone)
        return run_str_buckets(pl, keys_in, keys_out, vals_in, vals_out, tmp, stream);
    }
  }
  if constexpr (sizeof(K) == 8 && !std::is_same<Digit, DigitDiv64>::value) {
    if (pl.narrow) {
      // the passes move 4 bytes of key instead of 8: the first pass reads
      // the 8-byte keys and writes 32-bit words, the last writes 8-byte keys
      // back; a and b (within the alternate key array) hold the words
      uint32_t *a = (uint32_t *)(base + pl.off_keys_alt);
      uint32_t *b = (uint32_t *)(base + (pl.off_keys_alt + pl.n * 4 + 255) / 256 * 256);  // within n * 8 + 256
      return with_block<uint32_t, BITS>(pl.block, [&]<int BLOCK>() {
        return narrowed_passes<Digit, BITS, BLOCK>(
            pl, digits, pl.npasses, (const uint64_t *)keys_in, (uint64_t *)keys_out, vals_in, vals_out, a, b,
            pl.pairs ? (uint32_t *)(base + pl.off_vals_alt) : nullptr, pl.n, pl.ntiles,
            (uint32_t *)(base + pl.off_table), (uint32_t *)(base + pl.off_sums), stream);
      });
    }
  }
  return with_block<K, BITS>(pl.block, [&]<int BLOCK>() {
    return prescanned_passes<K, Digit, BITS, BLOCK, false>(
        pl, digits, pl.npasses, keys_in, keys_out, vals_in, vals_out, base + pl.off_keys_alt,
        pl.pairs ? (uint32_t *)(base + pl.off_vals_alt) : nullptr, pl.n, pl.ntiles,
        (uint32_t *)(base + pl.off_table), (uint32_t *)(base + pl.off_sums), nullptr, nullptr, stream);
  });
}

template <typename K, class Digit, int BITS>
static rs_status run_single(const Plan &pl, const Digit *digits, const void *ki, void *ko, const uint32_t *vi,
                            uint32_t *vo, void *tmp, hipStream_t s) {
  if (pl.prescanned) return run_prescanned<K, Digit, BITS>(pl, digits, ki, ko, vi, vo, tmp, s);
  return run_passes<K, Digit, BITS>(pl, digits, ki, ko, vi, vo, tmp, s);
}

template <typename K, class Digit>
static rs_status run_bits(const Plan &pl, const Digit *digits, const void *ki, void *ko, const uint32_t *vi,
                          uint32_t *vo, void *tmp, hipStream_t s) {
  if constexpr (sizeof(K) >= 16) {  // strings: 729 cells (base 27) or 256 (base 256) per pass
    if (pl.bits == 10) return run_single<K, Digit, 10>(pl, digits, ki, ko, vi, vo, tmp, s);
    if (pl.bits == 8) return run_single<K, Digit, 8>(pl, digits, ki, ko, vi, vo, tmp, s);
    return fail(RS_ERR_UNSUPPORTED, "string passes use 8- or 10-bit cells");
  }
  switch (pl.bits) {
  case 8:
    return run_single<K, Digit, 8>(pl, digits, ki, ko, vi, vo, tmp, s);
  case 10:
    return run_single<K, Digit, 10>(pl, digits, ki, ko, vi, vo, tmp, s);
  default:
    return run_single<K, Digit, 11>(pl, digits, ki, ko, vi, vo, tmp, s);
  }
}

static rs_status run_literal(const Plan &pl, const void *keys_in, void *keys_out, void *tmp, hipStream_t stream) {
  char *base = (char *)tmp;
  uint32_t *counts = (uint32_t *)(base + pl.off_counts);
  uint32_t *starts = (uint32_t *)(base + pl.off_starts);
  uint32_t *sums = (uint32_t *)(base + pl.off_sums);
  if (pl.map_rows > kMaxMapRows) return fail(RS_ERR_UNSUPPORTED, "too many traverse-map rows");
  RowMaps maps;
  maps.nlo = (uint32_t *)(base + pl.off_map_lo);
  maps.hi = (uint32_t *)(base + pl.off_map_hi);
  maps.rows = pl.map_rows;
  maps.inner = pl.map_inner;
  maps.by_inner = make_fastdiv32(pl.map_inner);
  rs_status st = launch_fill(counts, pl.ctrl_bytes, 0, stream);
  if (st != RS_OK) return st;
  // a few key rounds per workgroup so that the map merge stays small
  uint64_t blocks = (pl.n + 255) / 256;
  const uint64_t cap = (uint64_t)cu_count() * 4;
  if (blocks > cap) blocks = cap;
  const size_t map_lds = (size_t)2 * pl.map_rows * 4;  // per-workgroup row minima and maxima
  if (pl.key.key_bytes == 4)
    RS_TIMED("rs_cell_count", stream, hipLaunchKernelGGL((rs_cell_count<uint32_t, 256>), dim3((uint32_t)blocks), dim3(256), map_lds, stream,
                       (const uint32_t *)keys_in, pl.n, pl.literal_cells, counts, maps));
  else
    RS_TIMED("rs_cell_count", stream, hipLaunchKernelGGL((rs_cell_count<uint64_t, 256>), dim3((uint32_t)blocks), dim3(256), map_lds, stream,
                       (const uint64_t *)keys_in, pl.n, pl.literal_cells, counts, maps));
  if ((st = check_launch("rs_cell_count")) != RS_OK) return st;
  // reduce-then-scan over the cells (each down-sweep workgroup adds up the
  // chunk sums before its own, no spine launch); chunks that no row's
  // occupied range reaches are neither read nor written
  const uint64_t cells = pl.literal_cells;
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan_reduce<kScanBlock, kBigScanItems>), dim3(pl.scan_chunks), dim3(kScanBlock),
                              0, stream, counts, cells, nullptr, 1, sums, maps));
  RS_TIMED("rs_cell_scan", stream,
           hipLaunchKernelGGL((rs_cell_scan_down<kScanBlock, kBigScanItems, true>), dim3(pl.scan_chunks),
                              dim3(kScanBlock), 0,
                              stream, counts, cells, nullptr, 1, sums, starts, maps));
  if ((st = check_launch("rs_cell_scan")) != RS_OK) return st;
  const uint32_t eb = (pl.literal_cells + 255) / 256;
  if (pl.key.key_bytes == 4)
    RS_TIMED("rs_cell_emit", stream, hipLaunchKernelGGL((rs_cell_emit<uint32_t, 256>), dim3(eb), dim3(256), 0, stream, counts, starts,
                       pl.literal_cells, (uint32_t *)keys_out, pl.n, maps));
  else
    RS_TIMED("rs_cell_emit", stream, hipLaunchKernelGGL((rs_cell_emit<uint64_t, 256>), dim3(eb), dim3(256), 0, stream, counts, starts,
                       pl.literal_cells, (uint64_t *)keys_out, pl.n, maps));
  return check_launch("rs_cell_emit");
}

// ------------------------------------------------------------- validation

template <typename K>
__global__ __launch_bounds__(256) void rs_validate(const K *__restrict__ keys, uint64_t n, uint64_t space,
                                                   uint32_t *__restrict__ bad) {
  uint32_t mine = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256) {
    if constexpr (sizeof(K) == 16) {
      const Str16 k = keys[e];
      for (int w = 0; w < 4; ++w)
        for (int b = 0; b < 4; ++b) {
          const uint32_t byte = (k.w[w] >> (8 * b)) & 0xffu;
          mine += (byte != 0 && (byte < 'a' || byte > 'z')) ? 1u : 0u;
        }
    } else {
      mine += ((uint64_t)keys[e] >= space) ? 1u : 0u;
    }
  }
  mine = wave_sum(mine);
  if (lane_id() == 0 && mine) atomicAdd(bad, mine);
}

rs_status validate_keys(const Plan &pl, const void *keys, uint64_t n, void *tmp, hipStream_t s) {
  if (pl.key.is_signed) return RS_OK;  // every value of the type is a key
  if (pl.key.kind == RS_KEY_STR && pl.key.base == 256) return RS_OK;  // every byte is a symbol
  uint32_t *bad = (uint32_t *)tmp;
  if (hipMemsetAsync(bad, 0, 4, s) != hipSuccess) return fail(RS_ERR_HIP, "hipMemsetAsync");
  uint64_t blocks = (n + 255) / 256;
  if (blocks > (uint64_t)cu_count() * 8) blocks = (uint64_t)cu_count() * 8;
  // fixed point is signed: a negative key reads as a huge unsigned value
  const uint64_t space = pl.key.space ? pl.key.space : UINT64_MAX;
  switch (pl.key.key_bytes) {
  case 4:
    RS_TIMED("rs_validate", s, hipLaunchKernelGGL((rs_validate<uint32_t>), dim3((uint32_t)blocks), dim3(256), 0, s, (const uint32_t *)keys, n,
                       space, bad));
    break;
  case 8:
    RS_TIMED("rs_validate", s, hipLaunchKernelGGL((rs_validate<uint64_t>), dim3((uint32_t)blocks), dim3(256), 0, s, (const uint64_t *)keys, n,
                       pl.key.kind == RS_KEY_FIXED_I64 && space > (1ull << 63) ? (1ull << 63) : space, bad));
    break;
  default:
    RS_TIMED("rs_validate", s, hipLaunchKernelGGL((rs_validate<Str16>), dim3((uint32_t)blocks), dim3(256), 0, s, (const Str16 *)keys, n, 0,
                       bad));
  }
  rs_status st = check_launch("rs_validate");
  if (st != RS_OK) return st;
  uint32_t h = 0;
  if (hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(RS_ERR_HIP, "validation copy");
  if (h) return fail(RS_ERR_KEY_RANGE, std::to_string(h) + " keys outside the count space");
  return RS_OK;
}

rs_status check_alignment(const KeyInfo &k, const void *ki, const void *ko, const void *vi, const void *vo,
                          const void *tmp) {
  const uintptr_t kb = k.key_bytes;
  if ((uintptr_t)ki % kb || (uintptr_t)ko % kb)
    return fail(RS_ERR_UNSUPPORTED, "keys must be aligned to the key size (" + std::to_string(kb) + " bytes)");
  if ((uintptr_t)vi % 4 || (uintptr_t)vo % 4) return fail(RS_ERR_UNSUPPORTED, "values must be 4-byte aligned");
  if ((uintptr_t)tmp % 256) return fail(RS_ERR_UNSUPPORTED, "tmp must be 256-byte aligned");
  return RS_OK;
}

// A short array (at most kLocalMaxN keys): one workgroup loads it into LDS,
// runs every pass there and writes it back, so keys_out may equal keys_in.
template <typename K, class Digit>
static rs_status run_local(const Plan &pl, const Digit *digits, const void *ki, void *ko, const uint32_t *vi,
                           uint32_t *vo, hipStream_t s) {
  static_assert(256 * 16 == kLocalMaxN, "one tile of rs_local_sort");
  if (pl.n > kLocalMaxN) return fail(RS_ERR_UNSUPPORTED, "array too long for one workgroup");
  SmallParams<Digit> sp;
  memset(&sp, 0, sizeof sp);
  for (uint32_t i = 0; i < pl.npasses; ++i) {
    sp.digit[i] = digits[i];
    sp.pass_cells[i] = pl.pass_cells[i];
  }
  sp.npasses = pl.npasses;
  sp.single_n = pl.n;
  if (vi)
    RS_TIMED("rs_small_sort", s, hipLaunchKernelGGL((rs_local_sort<K, Digit, 256, 16, true>), dim3(1), dim3(256), 0, s,
                                                    sp, (const K *)ki, (K *)ko, vi, vo));
  else
    RS_TIMED("rs_small_sort", s, hipLaunchKernelGGL((rs_local_sort<K, Digit, 256, 16, false>), dim3(1), dim3(256), 0,
                                                    s, sp, (const K *)ki, (K *)ko, nullptr, nullptr));
  return check_launch("rs_local_sort");
}

rs_status run_plan(const Plan &pl, const void *ki, void *ko, const uint32_t *vi, uint32_t *vo, void *tmp,
                   hipStream_t s) {
  if (pl.n == 0) return RS_OK;
  if (pl.local) {
    switch (pl.mode) {
    case kModePow2:
      if (pl.key.key_bytes == 4) return run_local<uint32_t, DigitPow2>(pl, pl.p2, ki, ko, vi, vo, s);
      return run_local<uint64_t, DigitPow2>(pl, pl.p2, ki, ko, vi, vo, s);
    case kModeDiv32:
      if (pl.key.key_bytes == 4) return run_local<uint32_t, DigitDiv32>(pl, pl.d32, ki, ko, vi, vo, s);
      return run_local<uint64_t, DigitDiv32>(pl, pl.d32, ki, ko, vi, vo, s);
    case kModeDiv64:
      return run_local<uint64_t, DigitDiv64>(pl, pl.d64, ki, ko, vi, vo, s);
    default:
      return fail(RS_ERR_BAD_DESC, "short arrays of this key kind have no on-chip sort");
    }
  }
  if (pl.literal) return run_literal(pl, ki, ko, tmp, s);
  const uint32_t kb = pl.key.key_bytes;
  switch (pl.mode) {
  case kModePow2:
    if (kb == 4) return run_bits<uint32_t, DigitPow2>(pl, pl.p2, ki, ko, vi, vo, tmp, s);
    return run_bits<uint64_t, DigitPow2>(pl, pl.p2, ki, ko, vi, vo, tmp, s);
  case kModeDiv32:
    if (kb == 4) return run_bits<uint32_t, DigitDiv32>(pl, pl.d32, ki, ko, vi, vo, tmp, s);
    return run_bits<uint64_t, DigitDiv32>(pl, pl.d32, ki, ko, vi, vo, tmp, s);
  case kModeDiv64:
    return run_bits<uint64_t, DigitDiv64>(pl, pl.d64, ki, ko, vi, vo, tmp, s);
  case kModeStr16:
    return run_bits<Str16, DigitStr16>(pl, pl.s16, ki, ko, vi, vo, tmp, s);
  }
  return fail(RS_ERR_BAD_DESC, "unknown digit mode");
}

rs_status sort_common(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                      uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream, bool pairs) {
  g_last_error.clear();
  if (!desc) return fail(RS_ERR_NULL_ARG, "desc is NULL");
  if (n == 0) return RS_OK;
  if (!keys_in || !keys_out || !tmp) return fail(RS_ERR_NULL_ARG, "keys_in, keys_out and tmp are required");
  if (pairs && (!vals_in || !vals_out)) return fail(RS_ERR_NULL_ARG, "vals_in and vals_out are required");
  Plan pl;
  std::string why;
  rs_status st = make_plan(desc, n, pairs, current_tuning(desc, n, pairs), &pl, &why);
  if (st != RS_OK) return fail(st, why);
  if (tmp_bytes < pl.total)
    return fail(RS_ERR_TMP_TOO_SMALL, "tmp_bytes " + std::to_string(tmp_bytes) + " < " + std::to_string(pl.total));
  if ((st = check_alignment(pl.key, keys_in, keys_out, vals_in, vals_out, tmp)) != RS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (desc->flags & RS_FLAG_VALIDATE) {
    st = validate_keys(pl, keys_in, n, tmp, s);
    if (st != RS_OK) return st;
  }
  return run_plan(pl, keys_in, keys_out, vals_in, vals_out, tmp, s);
}


}  // namespace rs

using namespace rs;

extern "C" {

const char *rs_status_string(rs_status s) {
  switch (s) {
  case RS_OK: return "ok";
  case RS_ERR_NULL_ARG: return "null argument";
  case RS_ERR_BAD_DESC: return "bad key description";
  case RS_ERR_KEY_RANGE: return "key outside the count space";
  case RS_ERR_TMP_TOO_SMALL: return "scratch buffer too small";
  case RS_ERR_UNSUPPORTED: return "unsupported size or shape";
  case RS_ERR_OOM: return "out of host memory";
  case RS_ERR_HIP: return "HIP runtime error";
  case RS_ERR_BUSY: return "busy";
  }
  return "unknown status";
}

const char *rs_last_error(void) { return g_last_error.c_str(); }

rs_status rs_temp_bytes(const rs_key_desc *desc, uint64_t n, int with_values, size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(RS_ERR_NULL_ARG, "bytes is NULL");
  Plan pl;
  std::string why;
  rs_status st = make_plan(desc, n, with_values != 0, current_tuning(desc, n, with_values != 0), &pl, &why);
  if (st != RS_OK) return fail(st, why);
  *bytes = pl.total;
  return RS_OK;
}

rs_status rs_sort_keys(const rs_key_desc *desc, const void *keys_in, void *keys_out, uint64_t n, void *tmp,
                       size_t tmp_bytes, void *stream) {
  return sort_common(desc, keys_in, keys_out, nullptr, nullptr, n, tmp, tmp_bytes, stream, false);
}

rs_status rs_sort_pairs(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                        uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream) {
  return sort_common(desc, keys_in, keys_out, vals_in, vals_out, n, tmp, tmp_bytes, stream, true);
}

}  // extern "C"
