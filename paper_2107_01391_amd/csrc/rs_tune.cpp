// rs_tune.cpp -- tuning choices per (key description, size class), and the
// autotuner that measures them.
//
// A choice fixes how the digit dimensions are grouped into passes (bits per
// pass for power-of-two bases, the largest count space of a pass for other
// bases), the tile width of prescanned passes, and the size from which a
// single array uses prescanned rather than chained passes.  The sorted
// output does not depend on it (every grouping is a valid hierarchy of
// Section 2.2); only the time does.
//
// Precedence: a candidate being timed by the tuner (this thread only), then
// the environment variables (testing), then the kept choice of the size
// class, then the defaults:
//   RS_PRESCAN_MIN_N  single arrays from this length use prescanned passes
//   RS_DIGIT_BITS     bits of a pass for power-of-two bases (4..11)
//   RS_TILE_BLOCK     threads per tile of prescanned passes (256 or 512)
//   RS_MAX_CELLS      largest count space of one pass for other bases (2..2048)
#include "rs_tune.h"

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rs_internal.h"

namespace rs {

namespace {

using TuneKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, bool, bool, uint32_t>;

struct Table {
  std::mutex mu;
  std::map<TuneKey, Tuning> kept;
};

Table &table() {
  static Table *t = new Table();
  return *t;
}

thread_local const Tuning *t_override = nullptr;

uint32_t size_class(uint64_t n) {
  uint32_t c = 0;
  while (n > 1) {
    n >>= 1;
    ++c;
  }
  return c;
}

TuneKey key_of(const rs_key_desc *d, uint64_t n, bool pairs, bool batched) {
  return TuneKey(d->kind, d->base, d->ndims, d->frac_digits, d->str_width, pairs, batched, size_class(n));
}

uint64_t env_u64(const char *name, uint64_t dflt) {
  const char *v = getenv(name);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  unsigned long long x = strtoull(v, &end, 10);
  return (end && *end == 0) ? (uint64_t)x : dflt;
}

bool valid(const Tuning &t) {
  return t.digit_bits >= 4 && t.digit_bits <= 11 && t.max_cells >= 2 && t.max_cells <= 2048 &&
         (t.tile_block == 256 || t.tile_block == 512);
}

Tuning from_abi(const rs_tuning &a) {
  Tuning t;
  t.digit_bits = a.digit_bits;
  t.max_cells = a.max_cells;
  t.tile_block = a.tile_block;
  t.prescan_min_n = a.prescan_min_n;
  return t;
}

rs_tuning to_abi(const Tuning &t) {
  rs_tuning a;
  a.digit_bits = t.digit_bits;
  a.max_cells = t.max_cells;
  a.tile_block = t.tile_block;
  a.reserved = 0;
  a.prescan_min_n = t.prescan_min_n;
  return a;
}

// Candidate choices for a description: every distinct grouping of the
// digits into passes of at most 2048 cells, times both tile widths, times
// (single arrays) chained or prescanned passes.
std::vector<Tuning> candidates(const rs_key_desc *desc, uint64_t n, bool batched) {
  KeyInfo k;
  std::string why;
  std::vector<Tuning> out;
  if (key_info(desc, &k, &why) != RS_OK) return out;
  std::vector<Tuning> groupings;
  if (k.kind != RS_KEY_STR && k.pow2) {
    // d dimensions of m bits per pass: passes of 2^(d m) cells, 16..2048
    const uint32_t m = k.log2_base;
    for (uint32_t d = 1; d * m <= 11; ++d) {
      if (d * m < 4 && (d + 1) * m <= 11) continue;
      Tuning t;
      t.digit_bits = d * m < 4 ? 4 : d * m;
      groupings.push_back(t);
    }
  } else if (k.kind == RS_KEY_STR) {
    groupings.push_back(Tuning());  // two characters per pass, fixed
  } else {
    uint64_t cells = k.base;
    for (uint32_t w = 1; w <= k.ndims && cells <= 2048; ++w, cells *= k.base) {
      Tuning t;
      t.max_cells = (uint32_t)cells;
      groupings.push_back(t);
    }
  }
  const uint32_t blocks[2] = {256, 512};
  for (const Tuning &g : groupings)
    for (uint32_t b : blocks) {
      if (b == 512 && k.key_bytes > 8) continue;
      Tuning t = g;
      t.tile_block = b;
      if (batched) {
        out.push_back(t);
      } else {
        t.prescan_min_n = 1ull << size_class(n);  // prescanned for the whole class
        out.push_back(t);
        if (b == 256) {  // chained passes use 256-thread tiles only
          t.prescan_min_n = ~0ull;
          out.push_back(t);
        }
      }
    }
  return out;
}

struct OverrideScope {
  explicit OverrideScope(const Tuning *t) { t_override = t; }
  ~OverrideScope() { t_override = nullptr; }
};

// Times `run` (one warm-up, then reps) on the stream; < 0 on failure.
double time_runs(const std::function<rs_status()> &run, hipStream_t s, uint32_t reps) {
  if (run() != RS_OK) return -1.0;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  double ms = -1.0;
  bool ok = hipEventRecord(a, s) == hipSuccess;
  for (uint32_t r = 0; ok && r < reps; ++r) ok = run() == RS_OK;
  ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
  float f = 0.f;
  if (ok && hipEventElapsedTime(&f, a, b) == hipSuccess) ms = f / reps;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

rs_status tune_common(const rs_key_desc *desc, uint64_t n, bool pairs, bool batched,
                      const std::function<size_t()> &need, const std::function<rs_status()> &run, size_t tmp_bytes,
                      hipStream_t s, uint32_t reps, rs_tuning *best, double *best_ms) {
  if (reps == 0) reps = 3;
  const std::vector<Tuning> cands = candidates(desc, n, batched);
  if (cands.empty()) return fail(RS_ERR_BAD_DESC, "no candidate for this description");
  double best_t = -1.0;
  Tuning best_c;
  for (const Tuning &c : cands) {
    OverrideScope scope(&c);
    const size_t bytes = need();
    if (bytes == 0 || bytes > tmp_bytes) continue;  // tmp too small for this candidate
    const double ms = time_runs(run, s, reps);
    if (ms < 0) {
      if (hipStreamSynchronize(s) != hipSuccess) return fail(RS_ERR_HIP, "tuning run failed");
      continue;
    }
    if (best_t < 0 || ms < best_t) {
      best_t = ms;
      best_c = c;
    }
  }
  if (best_t < 0) return fail(RS_ERR_TMP_TOO_SMALL, "no candidate could run with this tmp");
  {
    Table &tb = table();
    std::lock_guard<std::mutex> g(tb.mu);
    tb.kept[key_of(desc, n, pairs, batched)] = best_c;
  }
  g_last_error.clear();
  if (best) *best = to_abi(best_c);
  if (best_ms) *best_ms = best_t;
  return RS_OK;
}

}  // namespace

Tuning current_tuning(const rs_key_desc *desc, uint64_t n, bool pairs, bool batched) {
  if (t_override) return *t_override;
  Tuning t;
  if (desc) {
    Table &tb = table();
    std::lock_guard<std::mutex> g(tb.mu);
    auto it = tb.kept.find(key_of(desc, n, pairs, batched));
    if (it != tb.kept.end()) t = it->second;
  }
  t.prescan_min_n = env_u64("RS_PRESCAN_MIN_N", t.prescan_min_n);
  const uint64_t cells = env_u64("RS_MAX_CELLS", t.max_cells);
  if (cells >= 2 && cells <= 2048) t.max_cells = (uint32_t)cells;
  const uint64_t block = env_u64("RS_TILE_BLOCK", t.tile_block);
  if (block == 256 || block == 512) t.tile_block = (uint32_t)block;
  const uint64_t bits = env_u64("RS_DIGIT_BITS", t.digit_bits);
  if (bits >= 4 && bits <= 11) t.digit_bits = (uint32_t)bits;
  return t;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_tuning_get(const rs_key_desc *desc, uint64_t n, int with_values, int batched, rs_tuning *out) {
  g_last_error.clear();
  if (!desc || !out) return fail(RS_ERR_NULL_ARG, "desc and out are required");
  *out = to_abi(current_tuning(desc, n, with_values != 0, batched != 0));
  return RS_OK;
}

rs_status rs_tuning_set(const rs_key_desc *desc, uint64_t n, int with_values, int batched, const rs_tuning *t) {
  g_last_error.clear();
  if (!desc || !t) return fail(RS_ERR_NULL_ARG, "desc and t are required");
  const Tuning c = from_abi(*t);
  if (!valid(c)) return fail(RS_ERR_BAD_DESC, "tuning field out of range");
  Table &tb = table();
  std::lock_guard<std::mutex> g(tb.mu);
  tb.kept[key_of(desc, n, with_values != 0, batched != 0)] = c;
  return RS_OK;
}

rs_status rs_tuning_clear(void) {
  g_last_error.clear();
  Table &tb = table();
  std::lock_guard<std::mutex> g(tb.mu);
  tb.kept.clear();
  return RS_OK;
}

rs_status rs_tune_temp_bytes(const rs_key_desc *desc, uint64_t n, uint32_t nseg, int with_values, size_t *bytes) {
  g_last_error.clear();
  if (!desc || !bytes) return fail(RS_ERR_NULL_ARG, "desc and bytes are required");
  size_t most = 0;
  for (const Tuning &c : candidates(desc, n, nseg != 0)) {
    OverrideScope scope(&c);
    size_t b = 0;
    const rs_status st = nseg ? rs_batched_temp_bytes(desc, n, nseg, with_values, &b)
                              : rs_temp_bytes(desc, n, with_values, &b);
    if (st == RS_OK && b > most) most = b;
  }
  if (most == 0) return fail(RS_ERR_BAD_DESC, "no candidate for this description");
  *bytes = most;
  g_last_error.clear();
  return RS_OK;
}

rs_status rs_tune_sort(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                       uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream, uint32_t reps,
                       rs_tuning *best, double *best_ms) {
  g_last_error.clear();
  if (!desc || !keys_in || !keys_out || !tmp) return fail(RS_ERR_NULL_ARG, "desc, keys and tmp are required");
  if (keys_in == keys_out || (vals_in && vals_in == vals_out))
    return fail(RS_ERR_UNSUPPORTED, "tuning needs outputs distinct from the inputs");
  if (n == 0) return fail(RS_ERR_UNSUPPORTED, "nothing to tune on");
  const bool pairs = vals_in != nullptr;
  hipStream_t s = (hipStream_t)stream;
  return tune_common(
      desc, n, pairs, false,
      [&]() {
        size_t b = 0;
        return rs_temp_bytes(desc, n, pairs, &b) == RS_OK ? b : (size_t)0;
      },
      [&]() {
        return pairs ? rs_sort_pairs(desc, keys_in, keys_out, vals_in, vals_out, n, tmp, tmp_bytes, s)
                     : rs_sort_keys(desc, keys_in, keys_out, n, tmp, tmp_bytes, s);
      },
      tmp_bytes, s, reps, best, best_ms);
}

rs_status rs_tune_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                          uint32_t *vals_out, const uint64_t *d_seg_offsets, uint32_t nseg, uint64_t total, void *tmp,
                          size_t tmp_bytes, void *stream, uint32_t reps, rs_tuning *best, double *best_ms) {
  g_last_error.clear();
  if (!desc || !keys_in || !keys_out || !tmp || !d_seg_offsets)
    return fail(RS_ERR_NULL_ARG, "desc, keys, offsets and tmp are required");
  if (keys_in == keys_out || (vals_in && vals_in == vals_out))
    return fail(RS_ERR_UNSUPPORTED, "tuning needs outputs distinct from the inputs");
  if (nseg == 0 || total == 0) return fail(RS_ERR_UNSUPPORTED, "nothing to tune on");
  const bool pairs = vals_in != nullptr;
  hipStream_t s = (hipStream_t)stream;
  return tune_common(
      desc, total, pairs, true,
      [&]() {
        size_t b = 0;
        return rs_batched_temp_bytes(desc, total, nseg, pairs, &b) == RS_OK ? b : (size_t)0;
      },
      [&]() {
        return rs_sort_batched(desc, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, nseg, total, tmp,
                               tmp_bytes, s);
      },
      tmp_bytes, s, reps, best, best_ms);
}

rs_status rs_tuning_save(const char *path) {
  g_last_error.clear();
  if (!path) return fail(RS_ERR_NULL_ARG, "path is NULL");
  FILE *f = fopen(path, "w");
  if (!f) return fail(RS_ERR_UNSUPPORTED, std::string("cannot write ") + path);
  Table &tb = table();
  std::lock_guard<std::mutex> g(tb.mu);
  fprintf(f, "# kind base ndims frac_digits str_width pairs batched size_class digit_bits max_cells tile_block "
             "prescan_min_n\n");
  for (const auto &kv : tb.kept) {
    const TuneKey &k = kv.first;
    const Tuning &t = kv.second;
    fprintf(f, "%u %u %u %u %u %d %d %u %u %u %u %llu\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), (int)std::get<5>(k), (int)std::get<6>(k), std::get<7>(k), t.digit_bits,
            t.max_cells, t.tile_block, (unsigned long long)t.prescan_min_n);
  }
  const bool ok = fclose(f) == 0;
  return ok ? RS_OK : fail(RS_ERR_UNSUPPORTED, std::string("cannot write ") + path);
}

rs_status rs_tuning_load(const char *path) {
  g_last_error.clear();
  if (!path) return fail(RS_ERR_NULL_ARG, "path is NULL");
  FILE *f = fopen(path, "r");
  if (!f) return fail(RS_ERR_UNSUPPORTED, std::string("cannot read ") + path);
  std::vector<std::pair<TuneKey, Tuning>> rows;
  char line[512];
  rs_status st = RS_OK;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    unsigned kind, base, ndims, frac, sw, cls, bits, cells, block;
    int pairs, batched;
    unsigned long long pmin;
    if (sscanf(line, "%u %u %u %u %u %d %d %u %u %u %u %llu", &kind, &base, &ndims, &frac, &sw, &pairs, &batched,
               &cls, &bits, &cells, &block, &pmin) != 12) {
      st = fail(RS_ERR_BAD_DESC, std::string("malformed tuning line: ") + line);
      break;
    }
    Tuning t;
    t.digit_bits = bits;
    t.max_cells = cells;
    t.tile_block = block;
    t.prescan_min_n = pmin;
    if (!valid(t)) {
      st = fail(RS_ERR_BAD_DESC, std::string("tuning field out of range: ") + line);
      break;
    }
    rows.emplace_back(TuneKey(kind, base, ndims, frac, sw, pairs != 0, batched != 0, cls), t);
  }
  fclose(f);
  if (st != RS_OK) return st;
  Table &tb = table();
  std::lock_guard<std::mutex> g(tb.mu);
  for (const auto &r : rows) tb.kept[r.first] = r.second;
  return RS_OK;
}

}  // extern "C"
