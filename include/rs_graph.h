/*
 * rs_graph.h -- sorts captured once as a HIP graph and replayed.
 *
 * The launch sequence of a sort depends only on its sizes (n; for the
 * batched form total and nseg), never on the key values, and every size
 * the kernels need beyond that is read on the device.  So a sort can be
 * captured once and replayed with one hipGraphLaunch.  Before each replay
 * the caller may rewrite the contents of the buffers: the keys, values and
 * segment offsets.  Replays see the new data provided the sizes stay the
 * same.
 *
 * The graph keeps the pointers it was made with.  The caller keeps every
 * buffer (inputs, outputs, offsets, tmp) alive and unmoved until
 * rs_graph_destroy.  Replays of one graph must not overlap: they share its
 * tmp.  RS_FLAG_VALIDATE is refused, because validation synchronises.
 */
#ifndef RS_GRAPH_H
#define RS_GRAPH_H

#include <stddef.h>
#include <stdint.h>

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_graph rs_graph;

/* Captures rs_sort_pairs (vals_in != NULL) or rs_sort_keys (vals_in and
 * vals_out NULL) with these arguments.  On success *out owns the graph. */
rs_status rs_graph_sort(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                        uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, rs_graph **out);

/* Captures rs_sort_batched with these arguments. */
rs_status rs_graph_sort_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out,
                                const uint32_t *vals_in, uint32_t *vals_out, const uint64_t *d_seg_offsets,
                                uint32_t nseg, uint64_t total, void *tmp, size_t tmp_bytes, rs_graph **out);

/* Enqueues one replay on `stream` (asynchronous). */
rs_status rs_graph_launch(rs_graph *g, void *stream);

/* Frees the graph (NULL is a no-op).  Pending replays must have completed. */
rs_status rs_graph_destroy(rs_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* RS_GRAPH_H */
