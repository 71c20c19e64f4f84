// rs_server.cpp -- continuous batching of sort requests (rs_server.h).
//
// State machine of a request: queued (admitted, copied into the arena) ->
// running (in a launch on one of the streams) -> done (its launch's event
// completed) -> released (arena range and slot free again).
//
// Threads: callers submit and release; one dispatcher thread forms launches
// whenever a stream is idle; one completion thread watches the launches'
// events.  One mutex guards all state.
#include "rs_server.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rs_internal.h"

namespace rs {
namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

enum ReqState { kQueued, kRunning, kDone };

struct Request {
  uint64_t offset = 0, n = 0;
  uint64_t arrival = 0, done_at = 0;
  ReqState state = kQueued;
  rs_status status = RS_OK;
};

struct Launch {
  uint32_t stream = 0;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> tickets;
};

struct Span {
  uint64_t offset, n;
};

// Scratch of one launch stream inside `work`.
struct StreamWork {
  size_t tmp_off = 0, tmp_bytes = 0, lo_off = 0, hi_off = 0;
};

struct Layout {
  size_t tmp_bytes = 0;
  std::vector<StreamWork> per;
  size_t total = 0;
};

rs_status check_config(const rs_key_desc *desc, const rs_server_config *c) {
  if (!desc || !c) return fail(RS_ERR_NULL_ARG, "desc and cfg are required");
  if (c->capacity == 0 || c->capacity > (1ull << 32)) return fail(RS_ERR_BAD_DESC, "capacity must be in [1, 2^32]");
  if (c->max_slots == 0 || c->max_slots > (1u << 20)) return fail(RS_ERR_BAD_DESC, "max_slots must be in [1, 2^20]");
  if (c->streams == 0 || c->streams > 8) return fail(RS_ERR_BAD_DESC, "streams must be in [1, 8]");
  if (c->mode != RS_SERVE_BATCHED && c->mode != RS_SERVE_PER_REQUEST) return fail(RS_ERR_BAD_DESC, "unknown mode");
  if (desc->flags & RS_FLAG_VALIDATE) return fail(RS_ERR_UNSUPPORTED, "the server does not validate keys");
  return RS_OK;
}

uint32_t batch_cap(const rs_server_config *c) {
  return c->max_batch == 0 || c->max_batch > c->max_slots ? c->max_slots : c->max_batch;
}

rs_status layout_of(const rs_key_desc *desc, const rs_server_config *c, Layout *L) {
  rs_status st = check_config(desc, c);
  if (st != RS_OK) return st;
  const bool pairs = c->with_values != 0;
  size_t tmp = 0;
  std::string why;
  if (c->mode == RS_SERVE_BATCHED) {
    Plan p;
    st = make_batched(desc, c->capacity, c->capacity, batch_cap(c), pairs, &p, &why);
    if (st != RS_OK) return fail(st, why);
    tmp = p.total;
  }
  // a lone request runs the single-array sort (in both modes): the largest
  // request, and the largest chained one (its look-back words grow with n)
  const uint64_t sizes[2] = {std::min<uint64_t>(c->capacity, RS_MAX_ELEMENTS),
                             std::min<uint64_t>(c->capacity, 3ull << 20)};
  for (uint64_t n : sizes) {
    size_t b = 0;
    if ((st = rs_temp_bytes(desc, n, pairs, &b)) != RS_OK) return st;
    tmp = std::max(tmp, b);
  }
  L->tmp_bytes = align256(tmp);
  L->per.resize(c->streams);
  size_t off = 0;
  const size_t bounds = align256((size_t)batch_cap(c) * 8);
  for (uint32_t i = 0; i < c->streams; ++i) {
    L->per[i].tmp_off = off;
    L->per[i].tmp_bytes = L->tmp_bytes;
    off += L->tmp_bytes;
    L->per[i].lo_off = off;
    off += bounds;
    L->per[i].hi_off = off;
    off += bounds;
  }
  L->total = off;
  return RS_OK;
}

}  // namespace
}  // namespace rs

using namespace rs;

struct rs_server {
  rs_key_desc desc{};
  rs_server_config cfg{};
  Plan key_plan;  // key size and kind
  int device = 0;
  char *kin = nullptr, *kout = nullptr;
  uint32_t *vin = nullptr, *vout = nullptr;
  char *work = nullptr;
  Layout lay;

  hipStream_t upload = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<uint64_t *> staging;  // pinned: [lo | hi] per stream
  std::vector<bool> stream_busy;
  std::vector<hipEvent_t> event_pool;

  std::mutex mu;
  std::condition_variable cv_dispatch, cv_done, cv_complete;
  bool stopping = false;
  std::thread dispatcher, completer;

  std::map<uint64_t, uint64_t> free_ranges;  // offset -> length
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;
  std::deque<Launch> inflight;
  std::deque<uint64_t> done_q;  // done, not yet collected
  uint64_t next_ticket = 1;
  uint32_t slots_used = 0;

  // statistics since the last reset
  std::vector<double> lat_ms;
  uint64_t keys_sorted = 0, launches = 0, busy = 0, first_arrival = 0, last_done = 0;

  bool alloc_range(uint64_t n, uint64_t *off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const uint64_t rest = it->second - n, at = it->first + n;
      free_ranges.erase(it);
      if (rest) free_ranges[at] = rest;
      return true;
    }
    return false;
  }

  void free_range(uint64_t off, uint64_t n) {
    if (n == 0) return;
    auto next = free_ranges.lower_bound(off);
    if (next != free_ranges.end() && off + n == next->first) {
      n += next->second;
      next = free_ranges.erase(next);
    }
    if (next != free_ranges.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_ranges[off] = n;
  }

  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  void finish(uint64_t t, rs_status st, uint64_t when) {
    auto it = reqs.find(t);
    if (it == reqs.end()) return;
    Request &r = it->second;
    r.state = kDone;
    r.status = st;
    r.done_at = when;
    done_q.push_back(t);
    if (st == RS_OK) {
      lat_ms.push_back((double)(when - std::min(when, r.arrival)) / 1e6);
      keys_sorted += r.n;
      if (!first_arrival || r.arrival < first_arrival) first_arrival = r.arrival;
      last_done = std::max(last_done, when);
    }
  }

  // Enqueues one launch on stream i for the given requests.  Runs without
  // the lock: it touches only stream i's resources and the spans given.
  rs_status launch(uint32_t i, const std::vector<Span> &spans, hipEvent_t uploaded) {
    hipStream_t s = streams[i];
    if (hipStreamWaitEvent(s, uploaded, 0) != hipSuccess) return fail(RS_ERR_HIP, "hipStreamWaitEvent");
    const StreamWork &w = lay.per[i];
    void *tmp = work + w.tmp_off;
    const bool pairs = cfg.with_values != 0;
    const size_t kb = key_plan.key.key_bytes;
    const uint32_t min_batch = cfg.min_batch ? cfg.min_batch : 4;
    if (cfg.mode == RS_SERVE_PER_REQUEST || spans.size() < min_batch) {
      // one launch sequence per request: the baseline, and small batches
      for (const Span &r : spans) {
        const size_t o = (size_t)r.offset;
        rs_status st = pairs ? rs_sort_pairs(&desc, kin + o * kb, kout + o * kb, vin + o, vout + o, r.n, tmp,
                                             w.tmp_bytes, s)
                             : rs_sort_keys(&desc, kin + o * kb, kout + o * kb, r.n, tmp, w.tmp_bytes, s);
        if (st != RS_OK) return st;
      }
      return RS_OK;
    }
    // batched: one segmented sequence over [lo, hi) ranges of the arena;
    // the host knows the sizes, so the tile bound counts only the arrays
    // too large to sort on chip, and an all-small batch launches no pass
    Plan p;
    std::string why;
    rs_status st = make_batched(&desc, 1, cfg.capacity, (uint32_t)spans.size(), pairs, &p, &why);
    if (st != RS_OK) return fail(st, why);
    uint64_t *lo = staging[i], *hi = staging[i] + batch_cap(&cfg);
    uint64_t large = 0, small = 0, nsmall = 0;
    for (size_t j = 0; j < spans.size(); ++j) {
      lo[j] = spans[j].offset;
      hi[j] = spans[j].offset + spans[j].n;
      if (spans[j].n > p.seg.small_max) {
        large += spans[j].n;
      } else {
        small += spans[j].n;
        ++nsmall;
      }
    }
    if (large > 1) {
      st = make_batched(&desc, large, cfg.capacity, (uint32_t)spans.size(), pairs, &p, &why);
      if (st != RS_OK) return fail(st, why);
    }
    p.seg.any_large = large > 0;
    p.seg.small_len = nsmall ? small / nsmall : 0;
    if (p.total > w.tmp_bytes) return fail(RS_ERR_TMP_TOO_SMALL, "server scratch below this batch's plan");
    const size_t nb = spans.size() * 8;
    uint64_t *dlo = (uint64_t *)(work + w.lo_off), *dhi = (uint64_t *)(work + w.hi_off);
    if (hipMemcpyAsync(dlo, lo, nb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dhi, hi, nb, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(RS_ERR_HIP, "hipMemcpyAsync of array bounds");
    return batched_run(p, kin, kout, pairs ? vin : nullptr, pairs ? vout : nullptr, dlo, dhi, tmp, s);
  }

  void dispatch_loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_dispatch.wait(lk, [&] {
        if (stopping) return true;
        if (queue.empty()) return false;
        return std::find(stream_busy.begin(), stream_busy.end(), false) != stream_busy.end();
      });
      if (stopping) return;
      const uint32_t i = (uint32_t)(std::find(stream_busy.begin(), stream_busy.end(), false) - stream_busy.begin());
      // per-request: the head alone.  Batched: while the queue is no longer
      // than the launch streams (latency matters), a large head runs alone
      // and only the run of small requests at the head is batched; with a
      // backlog (throughput matters) everything queued is batched.  Queue
      // order is kept.
      const bool backlog = queue.size() > cfg.streams;
      const uint64_t big = backlog ? ~0ull : (cfg.batch_max_n ? cfg.batch_max_n : (1ull << 20));
      const bool alone = cfg.mode == RS_SERVE_PER_REQUEST || reqs[queue.front()].n > big;
      uint32_t take = alone ? 1u : batch_cap(&cfg);
      if (!alone) {
        // fewer than min_batch small requests at the head: dispatch the head
        // alone, as the per-request server does, so that the others go to
        // the other idle streams instead of running one after another in
        // this launch
        const uint32_t min_batch = cfg.min_batch ? cfg.min_batch : 4;
        uint32_t run = 0;
        for (auto it = queue.begin(); it != queue.end() && run < min_batch && reqs[*it].n <= big; ++it) ++run;
        if (run < min_batch) take = 1;
      }
      std::vector<uint64_t> tickets;
      std::vector<Span> spans;
      while (!queue.empty() && tickets.size() < take) {
        const uint64_t t = queue.front();
        Request &r = reqs[t];
        if (!alone && r.n > big) break;
        queue.pop_front();
        r.state = kRunning;
        tickets.push_back(t);
        spans.push_back(Span{r.offset, r.n});
      }
      stream_busy[i] = true;
      hipEvent_t uploaded = take_event(), done = take_event();
      lk.unlock();
      // every request taken was uploaded (in stream order) before it was queued
      rs_status st = (uploaded && done) ? RS_OK : fail(RS_ERR_HIP, "hipEventCreate");
      if (st == RS_OK && hipEventRecord(uploaded, upload) != hipSuccess) st = fail(RS_ERR_HIP, "hipEventRecord");
      if (st == RS_OK) st = launch(i, spans, uploaded);
      if (st == RS_OK && hipEventRecord(done, streams[i]) != hipSuccess) st = fail(RS_ERR_HIP, "hipEventRecord");
      lk.lock();
      if (uploaded) event_pool.push_back(uploaded);  // the wait is enqueued: the event may be recorded again
      if (st != RS_OK) {
        const uint64_t t_now = now_ns();
        for (uint64_t t : tickets) finish(t, st, t_now);
        if (done) event_pool.push_back(done);
        stream_busy[i] = false;
        cv_done.notify_all();
        continue;
      }
      ++launches;
      inflight.push_back(Launch{i, done, std::move(tickets)});
      cv_complete.notify_one();
    }
  }

  void complete_loop() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_complete.wait(lk, [&] { return stopping || !inflight.empty(); });
      if (inflight.empty()) {
        if (stopping) return;
        continue;
      }
      bool any = false;
      for (auto it = inflight.begin(); it != inflight.end();) {
        const hipError_t q = hipEventQuery(it->done);
        if (q == hipErrorNotReady) {
          ++it;
          continue;
        }
        const uint64_t t_now = now_ns();
        const rs_status st = q == hipSuccess ? RS_OK : fail(RS_ERR_HIP, "launch failed on the device");
        for (uint64_t t : it->tickets) finish(t, st, t_now);
        stream_busy[it->stream] = false;
        event_pool.push_back(it->done);
        it = inflight.erase(it);
        any = true;
      }
      if (any) {
        cv_done.notify_all();
        cv_dispatch.notify_one();
      } else {
        // launches are in flight: poll again at once (a timed sleep lasts
        // tens of microseconds past its request, all of it added latency)
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      }
    }
  }
};

extern "C" {

rs_status rs_server_work_bytes(const rs_key_desc *desc, const rs_server_config *cfg, size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(RS_ERR_NULL_ARG, "bytes is NULL");
  Layout L;
  rs_status st = layout_of(desc, cfg, &L);
  if (st != RS_OK) return st;
  *bytes = L.total;
  return RS_OK;
}

rs_status rs_server_create(const rs_key_desc *desc, const rs_server_config *cfg, void *keys_in, void *keys_out,
                           uint32_t *vals_in, uint32_t *vals_out, void *work, size_t work_bytes, rs_server **out) {
  g_last_error.clear();
  if (!out) return fail(RS_ERR_NULL_ARG, "out is NULL");
  *out = nullptr;
  Layout L;
  rs_status st = layout_of(desc, cfg, &L);
  if (st != RS_OK) return st;
  if (!keys_in || !keys_out || !work) return fail(RS_ERR_NULL_ARG, "arenas and work are required");
  if (cfg->with_values && (!vals_in || !vals_out)) return fail(RS_ERR_NULL_ARG, "value arenas are required");
  if (work_bytes < L.total) return fail(RS_ERR_TMP_TOO_SMALL, "work below rs_server_work_bytes");
  rs_server *s = new (std::nothrow) rs_server;
  if (!s) return fail(RS_ERR_OOM, "rs_server");
  s->desc = *desc;
  s->cfg = *cfg;
  std::string why;
  if ((st = make_plan(desc, 1, true, Tuning(), &s->key_plan, &why)) != RS_OK) {
    delete s;
    return fail(st, why);
  }
  if ((st = check_alignment(s->key_plan.key, keys_in, keys_out, vals_in, vals_out, work)) != RS_OK) {
    delete s;
    return st;
  }
  s->kin = (char *)keys_in;
  s->kout = (char *)keys_out;
  s->vin = cfg->with_values ? vals_in : nullptr;
  s->vout = cfg->with_values ? vals_out : nullptr;
  s->work = (char *)work;
  s->lay = L;
  s->free_ranges[0] = cfg->capacity;
  bool ok = hipGetDevice(&s->device) == hipSuccess &&
            hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) == hipSuccess;
  for (uint32_t i = 0; ok && i < cfg->streams; ++i) {
    hipStream_t st_i = nullptr;
    uint64_t *pin = nullptr;
    ok = hipStreamCreateWithFlags(&st_i, hipStreamNonBlocking) == hipSuccess &&
         hipHostMalloc((void **)&pin, (size_t)2 * batch_cap(cfg) * 8, hipHostMallocDefault) == hipSuccess;
    if (st_i) s->streams.push_back(st_i);
    if (pin) s->staging.push_back(pin);
    s->stream_busy.push_back(false);
  }
  if (!ok) {
    rs_server_destroy(s);
    return fail(RS_ERR_HIP, "stream or pinned staging creation failed");
  }
  s->dispatcher = std::thread([s] { s->dispatch_loop(); });
  s->completer = std::thread([s] { s->complete_loop(); });
  *out = s;
  return RS_OK;
}

rs_status rs_server_submit(rs_server *s, const void *keys, const uint32_t *vals, uint64_t n, uint64_t arrival_ns,
                           void *src_stream, uint64_t *ticket) {
  g_last_error.clear();
  if (!s || !ticket) return fail(RS_ERR_NULL_ARG, "server and ticket are required");
  if (n && (!keys || (s->cfg.with_values && !vals))) return fail(RS_ERR_NULL_ARG, "keys (and values) are required");
  if (n > RS_MAX_ELEMENTS || n > s->cfg.capacity) return fail(RS_ERR_UNSUPPORTED, "request larger than the arena");
  const uint64_t arrival = arrival_ns ? arrival_ns : now_ns();
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stopping) return fail(RS_ERR_BUSY, "server stopping");
  uint64_t off = 0;
  if (s->slots_used >= s->cfg.max_slots || (n && !s->alloc_range(n, &off))) {
    ++s->busy;
    return fail(RS_ERR_BUSY, "no free slot or arena range");
  }
  const uint64_t t = s->next_ticket++;
  Request r;
  r.offset = off;
  r.n = n;
  r.arrival = arrival;
  ++s->slots_used;
  if (n == 0) {
    r.state = kDone;
    r.done_at = arrival;
    s->reqs[t] = r;
    s->done_q.push_back(t);
    *ticket = t;
    return RS_OK;
  }
  const size_t kb = s->key_plan.key.key_bytes;
  // the upload stream does not synchronise with other streams: it first
  // waits for what the producer has enqueued on src_stream (the writes of
  // the sources), so the copies read finished data
  hipEvent_t produced = s->take_event();
  bool ok = produced && hipEventRecord(produced, (hipStream_t)src_stream) == hipSuccess &&
            hipStreamWaitEvent(s->upload, produced, 0) == hipSuccess;
  if (produced) s->event_pool.push_back(produced);  // the wait is enqueued: the event may be recorded again
  if (ok) ok = hipMemcpyAsync(s->kin + off * kb, keys, n * kb, hipMemcpyDefault, s->upload) == hipSuccess;
  if (ok && s->cfg.with_values)
    ok = hipMemcpyAsync(s->vin + off, vals, n * 4, hipMemcpyDefault, s->upload) == hipSuccess;
  if (!ok) {
    s->free_range(off, n);
    --s->slots_used;
    return fail(RS_ERR_HIP, "copy into the arena failed");
  }
  s->reqs[t] = r;
  s->queue.push_back(t);
  *ticket = t;
  lk.unlock();
  s->cv_dispatch.notify_one();
  return RS_OK;
}

rs_status rs_server_poll(rs_server *s, uint64_t ticket, int *done) {
  g_last_error.clear();
  if (!s || !done) return fail(RS_ERR_NULL_ARG, "server and done are required");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RS_ERR_BAD_DESC, "unknown ticket");
  *done = it->second.state == kDone;
  return RS_OK;
}

rs_status rs_server_wait(rs_server *s, uint64_t ticket) {
  g_last_error.clear();
  if (!s) return fail(RS_ERR_NULL_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RS_ERR_BAD_DESC, "unknown ticket");
  s->cv_done.wait(lk, [&] {
    auto j = s->reqs.find(ticket);
    return j == s->reqs.end() || j->second.state == kDone;
  });
  auto j = s->reqs.find(ticket);
  if (j == s->reqs.end()) return fail(RS_ERR_BAD_DESC, "ticket released while waiting");
  return j->second.status == RS_OK ? RS_OK : fail(j->second.status, "request failed");
}

rs_status rs_server_collect(rs_server *s, uint64_t *tickets, uint32_t max, uint32_t *count, uint32_t wait_us) {
  g_last_error.clear();
  if (!s || !count || (max && !tickets)) return fail(RS_ERR_NULL_ARG, "server, tickets and count are required");
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait_us && s->done_q.empty())
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done_q.empty(); });
  uint32_t k = 0;
  while (k < max && !s->done_q.empty()) {
    const uint64_t t = s->done_q.front();
    s->done_q.pop_front();
    if (s->reqs.count(t)) tickets[k++] = t;  // skip tickets already released
  }
  *count = k;
  return RS_OK;
}

rs_status rs_server_result(rs_server *s, uint64_t ticket, uint64_t *offset, uint64_t *n) {
  g_last_error.clear();
  if (!s || !offset || !n) return fail(RS_ERR_NULL_ARG, "server, offset and n are required");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RS_ERR_BAD_DESC, "unknown ticket");
  if (it->second.state != kDone) return fail(RS_ERR_BUSY, "request not done");
  if (it->second.status != RS_OK) return fail(it->second.status, "request failed");
  *offset = it->second.offset;
  *n = it->second.n;
  return RS_OK;
}

rs_status rs_server_release(rs_server *s, uint64_t ticket) {
  g_last_error.clear();
  if (!s) return fail(RS_ERR_NULL_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(RS_ERR_BAD_DESC, "unknown ticket");
    if (it->second.state != kDone) return fail(RS_ERR_BUSY, "request not done");
    s->free_range(it->second.offset, it->second.n);
    --s->slots_used;
    s->reqs.erase(it);
  }
  s->cv_done.notify_all();
  return RS_OK;
}

rs_status rs_server_get_stats(rs_server *s, rs_server_stats *out) {
  g_last_error.clear();
  if (!s || !out) return fail(RS_ERR_NULL_ARG, "server and out are required");
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->completed = s->lat_ms.size();
  out->keys_sorted = s->keys_sorted;
  out->launches = s->launches;
  out->busy = s->busy;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const size_t i = (size_t)(q * (double)(v.size() - 1) + 0.5);
      return v[std::min(i, v.size() - 1)];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / (double)v.size();
    out->max_ms = v.back();
    out->span_ms = (double)(s->last_done - s->first_arrival) / 1e6;
  }
  return RS_OK;
}

rs_status rs_server_reset_stats(rs_server *s) {
  g_last_error.clear();
  if (!s) return fail(RS_ERR_NULL_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  s->lat_ms.clear();
  s->keys_sorted = s->launches = s->busy = s->first_arrival = s->last_done = 0;
  return RS_OK;
}

rs_status rs_server_clock(uint64_t *ns) {
  g_last_error.clear();
  if (!ns) return fail(RS_ERR_NULL_ARG, "ns is NULL");
  *ns = now_ns();
  return RS_OK;
}

rs_status rs_server_destroy(rs_server *s) {
  g_last_error.clear();
  if (!s) return RS_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->queue.clear();  // not yet launched: dropped
    s->cv_done.wait(lk, [&] { return s->inflight.empty(); });
    s->stopping = true;
  }
  s->cv_dispatch.notify_all();
  s->cv_complete.notify_all();
  if (s->dispatcher.joinable()) s->dispatcher.join();
  if (s->completer.joinable()) s->completer.join();
  if (s->upload) hipStreamSynchronize(s->upload);
  for (hipStream_t st : s->streams) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  if (s->upload) hipStreamDestroy(s->upload);
  for (uint64_t *p : s->staging) hipHostFree(p);
  for (hipEvent_t e : s->event_pool) hipEventDestroy(e);
  delete s;
  return RS_OK;
}

}  // extern "C"
