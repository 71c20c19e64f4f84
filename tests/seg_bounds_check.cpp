// Host check of the batched form's bound resolution (rs_seg_bounds.h), the
// arithmetic rs_seg_plan applies to the caller's offsets: valid arrays pass
// unchanged, and whatever the offsets hold every array stays inside the
// buffers and the tiles inside the scratch's bound.
#include <stdio.h>

#include <random>
#include <vector>

#include "rs_seg_bounds.h"

using namespace rs;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      if (fails++ < 20) printf("FAIL line %d: %s\n", __LINE__, #c); \
    }                                                              \
  } while (0)

// rs_seg_plan's walk over all arrays, sequentially: resolved [lo, lo + len)
// of every array and the large arrays' tile ranges.
struct Resolved {
  std::vector<uint64_t> lo, len;
  std::vector<TileRange> tiles;  // per array ({0, 0} for small ones)
};

static Resolved plan(const std::vector<uint64_t> &lo, const std::vector<uint64_t> &hi, uint64_t extent,
                     uint32_t small_max, uint32_t tile, uint32_t bound) {
  Resolved r;
  uint32_t run = 0;
  for (size_t s = 0; s < lo.size(); ++s) {
    SegBounds b = resolve_segment(lo[s], hi[s], extent);
    TileRange tr{0, 0};
    if (b.len > small_max) {
      const uint32_t want = (uint32_t)((b.len + tile - 1) / tile);
      tr = cut_tiles(run, want, bound);
      const uint64_t fits = (uint64_t)(tr.last - tr.first) * tile;
      if (b.len > fits) b.len = fits;
      run = cut_tiles(run, want, bound).last;
    }
    r.lo.push_back(b.lo);
    r.len.push_back(b.len);
    r.tiles.push_back(tr);
  }
  return r;
}

int main() {
  const uint64_t M = RS_MAX_ELEMENTS;
  // single arrays
  {
    SegBounds b = resolve_segment(10, 20, 100);
    CHECK(b.lo == 10 && b.len == 10);
    b = resolve_segment(20, 10, 100);  // reversed: empty
    CHECK(b.lo == 20 && b.len == 0);
    b = resolve_segment(90, 150, 100);  // past the end: cut
    CHECK(b.lo == 90 && b.len == 10);
    b = resolve_segment(150, 160, 100);  // wholly past the end: empty at the end
    CHECK(b.lo == 100 && b.len == 0);
    b = resolve_segment(0, ~0ull, ~0ull);  // longer than an array may be
    CHECK(b.lo == 0 && b.len == M);
    b = resolve_segment(~0ull, 0, 1000);
    CHECK(b.lo == 1000 && b.len == 0);
  }
  // tile cuts
  {
    TileRange t = cut_tiles(5, 3, 100);
    CHECK(t.first == 5 && t.last == 8);
    t = cut_tiles(98, 5, 100);
    CHECK(t.first == 98 && t.last == 100);
    t = cut_tiles(100, 5, 100);
    CHECK(t.first == 100 && t.last == 100);
    t = cut_tiles(0xffffffffull + 7, 0xffffffffu, 50);
    CHECK(t.first == 50 && t.last == 50);
  }
  // valid offsets pass unchanged; tile bound as the planner sizes it
  std::mt19937_64 rng(7);
  const uint32_t tile = 8192, small_max = 4096;
  for (int trial = 0; trial < 200; ++trial) {
    const uint32_t nseg = 1 + (uint32_t)(rng() % 300);
    std::vector<uint64_t> off(nseg + 1, 0);
    for (uint32_t i = 0; i < nseg; ++i) off[i + 1] = off[i] + (rng() % 4 == 0 ? rng() % 40000 : rng() % 9000);
    const uint64_t total = off[nseg];
    const uint64_t full = (total + tile - 1) / tile;
    uint64_t bound = full + (nseg < total / tile ? nseg : total / tile);
    if (bound == 0) bound = 1;
    std::vector<uint64_t> lo(off.begin(), off.end() - 1), hi(off.begin() + 1, off.end());
    Resolved r = plan(lo, hi, total, small_max, tile, (uint32_t)bound);
    uint32_t expect_first = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
      CHECK(r.lo[s] == lo[s] && r.len[s] == hi[s] - lo[s]);
      if (r.len[s] > small_max) {
        CHECK(r.tiles[s].first == expect_first);
        CHECK(r.tiles[s].last - r.tiles[s].first == (r.len[s] + tile - 1) / tile);
        expect_first = r.tiles[s].last;
      }
    }
  }
  // arbitrary offsets: in bounds, tiles within the bound, each array's
  // tiles cover its resolved keys
  for (int trial = 0; trial < 2000; ++trial) {
    const uint32_t nseg = 1 + (uint32_t)(rng() % 64);
    const uint64_t extent = 1 + rng() % 200000;
    const uint32_t bound = 1 + (uint32_t)(rng() % 40);
    std::vector<uint64_t> lo(nseg), hi(nseg);
    for (uint32_t s = 0; s < nseg; ++s) {
      const int k = (int)(rng() % 5);
      lo[s] = k == 0 ? rng() : rng() % (extent + 10);
      hi[s] = k == 1 ? rng() : (k == 2 ? lo[s] - rng() % 100 : lo[s] + rng() % 100000);
    }
    Resolved r = plan(lo, hi, extent, small_max, tile, bound);
    uint32_t prev_last = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
      CHECK(r.lo[s] <= extent && r.len[s] <= extent - r.lo[s] && r.len[s] <= M);
      if (r.tiles[s].last || r.tiles[s].first) {
        CHECK(r.tiles[s].first == prev_last && r.tiles[s].last <= bound);
        CHECK(r.len[s] <= (uint64_t)(r.tiles[s].last - r.tiles[s].first) * tile);
        prev_last = r.tiles[s].last;
      }
    }
  }
  if (fails) {
    printf("%d failures\n", fails);
    return 1;
  }
  printf("seg bounds ok\n");
  return 0;
}
