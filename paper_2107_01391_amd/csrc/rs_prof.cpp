// rs_prof.cpp -- event-pair timing of the library's kernel launches.
#include "rs_prof.h"

#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "rs_internal.h"

namespace rs {

namespace {

struct Record {
  const char *name;
  hipEvent_t a, b;
};

struct Profiler {
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<Record> records;
  std::vector<hipEvent_t> pool;

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto &r : records) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    records.clear();
  }
};

Profiler &prof() {
  static Profiler *p = new Profiler();  // never destroyed: events outlive static teardown order
  return *p;
}

}  // namespace

bool prof_on() { return prof().on.load(std::memory_order_relaxed); }

void *prof_begin(const char *name, hipStream_t s) {
  Profiler &p = prof();
  // launches being captured into a graph are not timed
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.on) return nullptr;
  Record r{name, p.take(), p.take()};
  if (!r.a || !r.b) return nullptr;
  hipEventRecord(r.a, s);
  p.records.push_back(r);
  return (void *)(uintptr_t)p.records.size();
}

void prof_end(void *token, hipStream_t s) {
  if (!token) return;
  Profiler &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  const size_t i = (size_t)(uintptr_t)token - 1;
  if (i < p.records.size()) hipEventRecord(p.records[i].b, s);
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_prof_enable(int enable) {
  Profiler &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (enable) p.recycle();
  p.on = enable != 0;
  return RS_OK;
}

rs_status rs_prof_query(const char *name, uint64_t *launches, double *total_ms) {
  if (!name || !launches || !total_ms) return fail(RS_ERR_NULL_ARG, "name, launches and total_ms are required");
  Profiler &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  uint64_t n = 0;
  double ms = 0;
  for (auto &r : p.records) {
    if (strcmp(r.name, name) != 0) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(RS_ERR_HIP, "hipEventSynchronize");
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(RS_ERR_HIP, "hipEventElapsedTime");
    ms += t;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  return RS_OK;
}

}  // extern "C"
