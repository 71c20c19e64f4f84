// rs_graph.cpp -- capture of a sort's launch sequence into a HIP graph.
#include "rs_graph.h"

#include <functional>

#include "rs_internal.h"

struct rs_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace rs {

// Runs `body` on a private stream in capture mode and instantiates what it
// enqueued.  The capture is thread-local, so other threads' HIP calls are
// unaffected.
static rs_status capture(const std::function<rs_status(hipStream_t)> &body, rs_graph **out) {
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(RS_ERR_HIP, "hipStreamCreate");
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(s);
    return fail(RS_ERR_HIP, "hipStreamBeginCapture");
  }
  const rs_status st = body(s);
  const std::string why = g_last_error;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  hipStreamDestroy(s);
  if (st != RS_OK) {
    if (graph) hipGraphDestroy(graph);
    return fail(st, why);
  }
  if (e != hipSuccess || !graph) return fail(RS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(graph);
    return fail(RS_ERR_HIP, "hipGraphInstantiate");
  }
  rs_graph *g = new (std::nothrow) rs_graph;
  if (!g) {
    hipGraphExecDestroy(exec);
    hipGraphDestroy(graph);
    return fail(RS_ERR_OOM, "rs_graph");
  }
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return RS_OK;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_graph_sort(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                        uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, rs_graph **out) {
  g_last_error.clear();
  if (!out) return fail(RS_ERR_NULL_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(RS_ERR_NULL_ARG, "desc is NULL");
  if (desc->flags & RS_FLAG_VALIDATE) return fail(RS_ERR_UNSUPPORTED, "validation cannot be captured");
  return capture(
      [&](hipStream_t s) {
        return vals_in ? rs_sort_pairs(desc, keys_in, keys_out, vals_in, vals_out, n, tmp, tmp_bytes, s)
                       : rs_sort_keys(desc, keys_in, keys_out, n, tmp, tmp_bytes, s);
      },
      out);
}

rs_status rs_graph_sort_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out,
                                const uint32_t *vals_in, uint32_t *vals_out, const uint64_t *d_seg_offsets,
                                uint32_t nseg, uint64_t total, void *tmp, size_t tmp_bytes, rs_graph **out) {
  g_last_error.clear();
  if (!out) return fail(RS_ERR_NULL_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(RS_ERR_NULL_ARG, "desc is NULL");
  if (desc->flags & RS_FLAG_VALIDATE) return fail(RS_ERR_UNSUPPORTED, "validation cannot be captured");
  return capture(
      [&](hipStream_t s) {
        return rs_sort_batched(desc, keys_in, keys_out, vals_in, vals_out, d_seg_offsets, nseg, total, tmp,
                               tmp_bytes, s);
      },
      out);
}

rs_status rs_graph_launch(rs_graph *g, void *stream) {
  g_last_error.clear();
  if (!g) return fail(RS_ERR_NULL_ARG, "graph is NULL");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RS_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return RS_OK;
}

rs_status rs_graph_destroy(rs_graph *g) {
  g_last_error.clear();
  if (!g) return RS_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return RS_OK;
}

}  // extern "C"
