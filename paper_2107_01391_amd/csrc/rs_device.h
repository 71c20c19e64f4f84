// rs_device.h -- device building blocks of the gfx950 Recombinant Sort path.
//
// Digit codecs (the paper's hash of a key to the coordinates of its cell,
// Section 3.1.1 eq. (1)), wave64 helpers for stable in-wave ranking, block
// scans and the flag-tagged words of the decoupled look-back scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int kWave = 64;
constexpr int kMaxPasses = 16;
constexpr uint32_t kLdsCountBudget = 48 * 1024;  // bytes of LDS count tables per workgroup

// ------------------------------------------------------------- integer codec

// Division by an invariant divisor d >= 1 with one multiply-high, following
// Granlund & Montgomery, "Division by invariant integers using
// multiplication" (PLDI 1994), Figure 4.1: with l = ceil(log2 d) and
// m = floor(2^W (2^l - d) / d) + 1, q = (t + ((x - t) >> 1)) >> (l - 1)
// where t = mulhi(m, x).  Exact for every W-bit x.  d == 1 uses m = 0 and no
// shifts.
struct FastDiv32 {
  uint32_t m, s1, s2;
  __host__ __device__ __forceinline__ uint32_t div(uint32_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(m, x);
#else
    uint32_t t = (uint32_t)(((uint64_t)m * x) >> 32);
#endif
    return (t + ((x - t) >> s1)) >> s2;
  }
};

struct FastDiv64 {
  uint64_t m;
  uint32_t s1, s2;
  __host__ __device__ __forceinline__ uint64_t div(uint64_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t t = __umul64hi(m, x);
#else
    uint64_t t = (uint64_t)(((unsigned __int128)m * x) >> 64);
#endif
    return (t + ((x - t) >> s1)) >> s2;
  }
};

inline FastDiv32 make_fastdiv32(uint32_t d) {
  FastDiv32 f{0, 0, 0};
  if (d <= 1) return f;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  f.s1 = 1;
  f.s2 = l - 1;
  return f;
}

inline FastDiv64 make_fastdiv64(uint64_t d) {
  FastDiv64 f{0, 0, 0};
  if (d <= 1) return f;
  uint32_t l = 0;
  while (l < 64 && ((unsigned __int128)1 << l) < d) ++l;
  unsigned __int128 num = ((unsigned __int128)1 << 64) * (((unsigned __int128)1 << l) - d);
  f.m = (uint64_t)(num / d + 1);
  f.s1 = 1;
  f.s2 = l - 1;
  return f;
}

// 16-byte fixed-width string key.
struct alignas(16) Str16 {
  uint32_t w[4];
};

// One pass's cell of a key: the group of dimensions [lo, lo + width) counted
// from the least significant digit, as one row-major index in [0, b^width).
// Every codec first adds `bias` to the key (signed keys: 2^31 or 2^63, which
// maps the signed order onto the unsigned one; else 0) and, for descending
// order, complements the cell: cells - 1 - cell, written (cell ^ cx) + ca
// with (cx, ca) = (~0, cells), or (0, 0) ascending.
//
// Power-of-two base: a shift and a mask (descending: xor with the mask).
struct DigitPow2 {
  uint32_t shift, mask;
  uint32_t flip;  // mask when descending, else 0
  uint64_t bias;
  __host__ __device__ __forceinline__ uint32_t operator()(uint32_t v) const {
    return (((v + (uint32_t)bias) >> shift) & mask) ^ flip;
  }
  __host__ __device__ __forceinline__ uint32_t operator()(uint64_t v) const {
    return ((uint32_t)((v + bias) >> shift) & mask) ^ flip;
  }
};

// Any base, values below 2^32: (v / b^lo) mod b^width with two invariant
// divisions.  Used for 32-bit keys and for 64-bit keys whose whole space fits
// in 32 bits (their high word is zero for every key inside the space).
struct DigitDiv32 {
  FastDiv32 by_lo, by_cells;
  uint32_t cells;
  uint32_t cx, ca;  // descending complement
  uint64_t bias;
  __host__ __device__ __forceinline__ uint32_t operator()(uint32_t v) const {
    v += (uint32_t)bias;
    const uint32_t q = by_lo.div(v);
    return ((q - by_cells.div(q) * cells) ^ cx) + ca;
  }
  __host__ __device__ __forceinline__ uint32_t operator()(uint64_t v) const { return (*this)((uint32_t)v); }
};

// Any base, 64-bit values.
struct DigitDiv64 {
  FastDiv64 by_lo, by_cells;
  uint32_t cells;
  uint32_t cx, ca;  // descending complement
  uint64_t bias;
  __host__ __device__ __forceinline__ uint32_t operator()(uint64_t v) const {
    v += bias;
    const uint64_t q = by_lo.div(v);
    return ((uint32_t)(q - by_cells.div(q) * cells) ^ cx) + ca;
  }
};

// Strings: one dimension per byte; the group is the `width` symbols starting
// at byte `pos`, most significant first.  Base 27: pad (0) -> 0 and
// 'a'..'z' -> 1..26.  Base 256: the byte itself (memcmp order of any bytes).
struct DigitStr16 {
  uint32_t pos, width;
  uint32_t cx, ca;  // descending complement
  uint32_t base;    // 27 or 256
  __host__ __device__ __forceinline__ uint32_t operator()(const Str16 &k) const {
    uint64_t lo = (uint64_t)k.w[0] | ((uint64_t)k.w[1] << 32);
    uint64_t hi = (uint64_t)k.w[2] | ((uint64_t)k.w[3] << 32);
    uint32_t cell = 0;
    for (uint32_t i = 0; i < width; ++i) {
      uint32_t j = pos + i;
      uint32_t byte = (uint32_t)((j < 8 ? (lo >> (8 * j)) : (hi >> (8 * (j - 8)))) & 0xffu);
      if (base == 256) {
        cell = cell * 256u + byte;
      } else {
        // 'a'..'z' -> 1..26; a byte outside the alphabet (invalid input) is
        // clamped into the space so it can never index past the tables
        uint32_t sym = byte ? (byte - 96u < 26u ? byte - 96u : 26u) : 0u;
        cell = cell * 27u + sym;
      }
    }
    return (cell ^ cx) + ca;
  }
};

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

// ---------------------------------------------------------------- wave64 ops

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of `active` whose value d equals this lane's, from BITS ballots (one
// per bit of d).  Invalid lanes must not be in `active`.
// The lanes that agree with this one on bit b are ~(ballot ^ s), where s is
// this lane's bit spread over the word (0 or ~0): per bit a shift, a compare,
// a shift back and two logic ops per half of the mask (three-input ones
// where the compiler merges), with no per-lane select.  The ranking is bound
// by instruction issue, so this form, about 40% fewer instructions than
// selecting ballot or ~ballot per lane, shortens the scatter by about 9%.
template <int BITS>
__device__ __forceinline__ uint64_t match_any(uint32_t d, uint64_t active) {
  uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const uint32_t s = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
    const uint64_t v = ballot(s != 0);
    lo &= ~((uint32_t)v ^ s);
    hi &= ~((uint32_t)(v >> 32) ^ s);
  }
  return (uint64_t)hi << 32 | lo;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Exclusive scan, in place, of a[0..count) held in LDS by all BLOCK threads.
// wsum is LDS scratch of BLOCK/64 words.  Returns the total to every thread.
template <int BLOCK>
__device__ uint32_t block_exclusive_scan(uint32_t *a, uint32_t count, uint32_t *wsum) {
  constexpr int kWaves = BLOCK / kWave;
  const uint32_t t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const uint32_t per = (count + BLOCK - 1) / BLOCK;
  const uint32_t lo = t * per < count ? t * per : count;
  const uint32_t hi = lo + per < count ? lo + per : count;
  uint32_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += a[i];
  uint32_t incl = wave_inclusive_scan(s);
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    uint32_t v = wsum[w];
    before += (uint32_t)w < wave ? v : 0u;
    total += v;
  }
  uint32_t run = before + incl - s;
  for (uint32_t i = lo; i < hi; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

// ------------------------------------------------------ look-back words
//
// A 32-bit status word per (tile, cell): bits 31..30 flag, 29..0 value.
// flag 0 = not yet published, 1 = the tile's own count, 2 = inclusive prefix
// over every earlier tile.  Stored and loaded with agent-scope atomics so
// they are coherent across the XCDs' separate L2 caches.
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagPrefix = 2u << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1;

__device__ __forceinline__ void publish(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t peek(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the counts of every tile before `tile` (down to `first`) at column
// stride `stride`, walking back until a tile with an inclusive prefix.
__device__ __forceinline__ uint32_t look_back(const uint32_t *status, uint64_t tile, uint64_t first,
                                              uint64_t stride) {
  uint32_t excl = 0;
  uint64_t p = tile;
  while (p > first) {
    --p;
    uint32_t s;
    while (((s = peek(status + p * stride)) >> 30) == 0) __builtin_amdgcn_s_sleep(1);
    excl += s & kValueMask;
    if (s & kFlagPrefix) break;
  }
  return excl;
}

// Non-temporal loads for the count kernels' 16-byte reads of the keys
// (read once, nothing reused).  Measured on MI355X: a streaming read rises
// from 6.2 to 7.0 TB/s with the hint and the per-tile count of 2^28 u32
// keys from 0.25 to 0.20 ms; the scatter's loads and stores, and the
// batched form's one-key-per-lane count loads, are faster without it.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  if constexpr (sizeof(T) == 16) {
    const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    T r;
    __builtin_memcpy(&r, &x, 16);
    return r;
  } else {
    return __builtin_nontemporal_load(p);
  }
}

__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Counts value d into an LDS table held in `copies` copies (a power of two,
// `cstride` words apart): lane l adds to copy l % copies, so lanes of one
// wave that hold the same cell (skewed data, padding) serialise at most
// 64 / copies deep, with no ballot or compare on the way.
__device__ __forceinline__ void lds_count(uint32_t *table, uint32_t cstride, uint32_t copies, uint32_t d,
                                          bool valid) {
  if (valid) lds_add(table + (lane_id() & (copies - 1)) * cstride + d, 1u);
}

// Copies of an LDS count table that fit `budget` bytes (power of two, <= 8).
__host__ __device__ inline uint32_t count_copies(uint32_t words, uint32_t budget) {
  uint32_t c = 8;
  while (c > 1 && (uint64_t)c * (words + 1) * 4 > budget) c >>= 1;
  return c;
}

#endif  // device

}  // namespace rs
