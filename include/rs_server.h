/*
 * rs_server.h -- a served request loop over the sort: continuous batching of
 * independent sort requests on one GPU.
 *
 * Requests are independent arrays. This is bucket sort's independence of
 * buckets (Section 2.2): they need no order between them, so requests that
 * arrive while others run can be sorted together.
 *
 * Admission and placement:
 *   - A request is admitted only when it fits.  It needs a free range of the
 *     caller-provided device arena (admission by free HBM) and a free slot.
 *     Otherwise rs_server_submit returns RS_ERR_BUSY and the caller retries
 *     later.
 *   - On admission its keys (and values) are copied into the arena.
 *   - The sorted result appears at the same positions of the output arena.
 *     It stays there until the caller releases the request.
 *
 * Dispatch.  A dispatcher thread launches work whenever one of `streams`
 * launch streams is idle:
 *   - RS_SERVE_BATCHED: queued requests (up to max_batch) in one segmented
 *     launch sequence, the rs_sort_batched kernels over begin/end ranges of
 *     the arena.  While the queue holds no more requests than there are
 *     streams, a request of more than batch_max_n keys at the head runs
 *     alone and only the small requests at the head are batched, so small
 *     requests do not wait for a large one's sort; with a longer queue
 *     everything is batched.  With fewer than min_batch small requests at
 *     the head, the head alone is dispatched as a single-array sort (the
 *     others go to other idle streams), so light load runs as the
 *     baseline does.
 *   - RS_SERVE_PER_REQUEST: one rs_sort_pairs / rs_sort_keys launch per
 *     request (the baseline).
 *   - With streams > 1, launches overlap on the device.
 *
 * Completion.  A completion thread marks a request done once its launch's
 * event has completed.  The request's latency runs from its arrival (given
 * at submit, or the submit time) to that moment.  While launches are in
 * flight the thread polls their events without sleeping (it occupies one
 * host core then); with none in flight it blocks.
 *
 * Each request's result is the stable sort of its own keys.  It is the same
 * whichever other requests share its launch.
 *
 * All functions are thread-safe.  Device pointers belong to the current
 * device at rs_server_create.  The caller keeps every buffer passed to
 * rs_server_create alive until rs_server_destroy returns.
 */
#ifndef RS_SERVER_H
#define RS_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_server rs_server;

enum { RS_SERVE_BATCHED = 0, RS_SERVE_PER_REQUEST = 1 };

typedef struct rs_server_config {
  uint64_t capacity;     /* arena size in keys (at most 2^32) */
  uint32_t max_slots;    /* requests admitted at once: queued, running or not yet released */
  uint32_t max_batch;    /* most requests in one batched launch (0 = max_slots) */
  uint32_t streams;      /* launches in flight at once, 1..8 */
  uint32_t mode;         /* RS_SERVE_BATCHED or RS_SERVE_PER_REQUEST */
  uint32_t with_values;  /* requests carry uint32 values */
  uint32_t min_batch;    /* batched mode: fewest small requests at the head of the queue that are
                            batched; with fewer, the head is dispatched alone (0 = 4) */
  uint64_t batch_max_n;  /* batched mode, short queue: requests of more keys run alone (0 = 2^20) */
} rs_server_config;

typedef struct rs_server_stats {
  uint64_t completed;    /* requests done since the last reset */
  uint64_t keys_sorted;  /* their keys */
  uint64_t launches;     /* launch sequences issued */
  uint64_t busy;         /* submissions refused with RS_ERR_BUSY */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* latency: arrival to sorted */
  double span_ms;        /* first arrival to last completion */
} rs_server_stats;

/* Device scratch the server needs (`work`): per launch stream, the sort's
 * scratch at the arena's full size plus the array bounds of one batch. */
rs_status rs_server_work_bytes(const rs_key_desc *desc, const rs_server_config *cfg, size_t *bytes);

/* Starts a server.  keys_in / keys_out: arenas of cfg->capacity keys;
 * vals_in / vals_out: arenas of cfg->capacity uint32 values (NULL when
 * with_values is 0); work: rs_server_work_bytes bytes, 256-byte aligned.
 * All device memory, owned by the caller.  RS_FLAG_VALIDATE is refused. */
rs_status rs_server_create(const rs_key_desc *desc, const rs_server_config *cfg, void *keys_in, void *keys_out,
                           uint32_t *vals_in, uint32_t *vals_out, void *work, size_t work_bytes, rs_server **out);

/* Submits a request of n keys (and values when the server carries them).
 * keys / vals are host or device pointers.  The copy into the arena is
 * enqueued on the server's own upload stream and reads them later, so they
 * must stay allocated and unchanged until the request is done (a framework
 * allocator must not hand their memory to another tensor before then).
 * src_stream (a hipStream_t as void*, NULL = the null stream) is the stream
 * on which the sources were written: the upload first waits for the work
 * enqueued there before this call.  arrival_ns: the request's arrival on
 * rs_server_clock (0 = now).  RS_ERR_BUSY: not admitted now, nothing kept. */
rs_status rs_server_submit(rs_server *s, const void *keys, const uint32_t *vals, uint64_t n, uint64_t arrival_ns,
                           void *src_stream, uint64_t *ticket);

/* *done = 1 when the request is sorted (or failed: rs_server_wait returns
 * its status). */
rs_status rs_server_poll(rs_server *s, uint64_t ticket, int *done);

/* Blocks until the request is done; returns its status. */
rs_status rs_server_wait(rs_server *s, uint64_t ticket);

/* Moves up to `max` tickets of requests that finished since the last
 * collect (sorted or failed) into tickets[], in completion order, and sets
 * *count.  With wait_us > 0 and none ready, waits up to that long for one. */
rs_status rs_server_collect(rs_server *s, uint64_t *tickets, uint32_t max, uint32_t *count, uint32_t wait_us);

/* Where a done request's result lies: keys_out[*offset, *offset + *n) and
 * the same range of vals_out. */
rs_status rs_server_result(rs_server *s, uint64_t ticket, uint64_t *offset, uint64_t *n);

/* Frees a done request's arena range and slot. */
rs_status rs_server_release(rs_server *s, uint64_t ticket);

rs_status rs_server_get_stats(rs_server *s, rs_server_stats *out);
rs_status rs_server_reset_stats(rs_server *s);

/* The server's clock (steady, nanoseconds) for arrival times. */
rs_status rs_server_clock(uint64_t *ns);

/* Waits for launched work, stops the threads and frees the server (NULL is
 * a no-op).  Requests not yet launched are dropped. */
rs_status rs_server_destroy(rs_server *s);

#ifdef __cplusplus
}
#endif

#endif /* RS_SERVER_H */
