// Host check of the device codecs in rs_device.h: invariant division and the
// cell extraction of every digit mode, against plain arithmetic.
#include <stdio.h>
#include <stdlib.h>

#include <random>

#include "rs_device.h"

using namespace rs;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      if (fails++ < 20) printf("FAIL line %d: %s\n", __LINE__, #c); \
    }                                                              \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  const uint32_t divs32[] = {1, 2, 3, 7, 10, 27, 100, 729, 1000, 19683, 65536, 100000, 1000000, 999999937u,
                             (1u << 31) + 1, 0xffffffffu};
  for (uint32_t d : divs32) {
    FastDiv32 f = make_fastdiv32(d);
    const uint32_t edge[] = {0, 1, d - 1, d, d + 1, 2 * d - 1, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu};
    for (uint32_t x : edge) CHECK(f.div(x) == x / d);
    for (int i = 0; i < 200000; ++i) {
      uint32_t x = (uint32_t)rng();
      CHECK(f.div(x) == x / d);
    }
  }
  const uint64_t divs64[] = {1, 3, 10, 1000, 1000000, 1000000000ull, 1000000000000ull, 10000000000000000000ull,
                             (1ull << 63) + 5, 0xffffffffffffffffull, 27ull * 27 * 27 * 27 * 27 * 27 * 27};
  for (uint64_t d : divs64) {
    FastDiv64 f = make_fastdiv64(d);
    const uint64_t edge[] = {0, 1, d - 1, d, d + 1, 0x7fffffffffffffffull, 0xffffffffffffffffull};
    for (uint64_t x : edge) CHECK(f.div(x) == x / d);
    for (int i = 0; i < 200000; ++i) {
      uint64_t x = rng() >> (rng() % 64);
      CHECK(f.div(x) == x / d);
    }
  }
  // base-10 groups of three digits of a 9-digit fixed-point value
  for (uint32_t lo = 0; lo < 9; lo += 3) {
    uint32_t below = 1;
    for (uint32_t j = 0; j < lo; ++j) below *= 10;
    DigitDiv32 g{make_fastdiv32(below), make_fastdiv32(1000), 1000};
    DigitDiv64 h{make_fastdiv64(below), make_fastdiv64(1000), 1000};
    for (int i = 0; i < 100000; ++i) {
      uint64_t v = rng() % 1000000000ull;
      CHECK(g((uint64_t)v) == (v / below) % 1000);
      CHECK(h(v) == (v / below) % 1000);
    }
  }
  // power-of-two digits
  for (uint32_t shift = 0; shift < 32; shift += 8) {
    DigitPow2 p{shift, 255};
    for (int i = 0; i < 1000; ++i) {
      uint32_t v = (uint32_t)rng();
      CHECK(p(v) == ((v >> shift) & 255));
    }
  }
  // strings: two symbols per cell, pad sorts first
  for (int i = 0; i < 20000; ++i) {
    Str16 k;
    unsigned char b[16];
    int len = 1 + (int)(rng() % 16);
    for (int j = 0; j < 16; ++j) b[j] = j < len ? (unsigned char)('a' + rng() % 26) : 0;
    for (int w = 0; w < 4; ++w)
      k.w[w] = (uint32_t)b[4 * w] | ((uint32_t)b[4 * w + 1] << 8) | ((uint32_t)b[4 * w + 2] << 16) |
               ((uint32_t)b[4 * w + 3] << 24);
    for (uint32_t pos = 0; pos < 16; pos += 2) {
      DigitStr16 s{pos, 2};
      uint32_t s0 = b[pos] ? b[pos] - 'a' + 1 : 0, s1 = b[pos + 1] ? b[pos + 1] - 'a' + 1 : 0;
      CHECK(s(k) == s0 * 27 + s1);
    }
  }
  if (fails) {
    printf("%d failures\n", fails);
    return 1;
  }
  printf("codec ok\n");
  return 0;
}
