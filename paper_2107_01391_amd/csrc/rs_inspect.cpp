// rs_inspect.cpp -- rs_plan_inspect: the planner's choice, reported.
#include "rs_inspect.h"

#include <string>

#include "rs_internal.h"

extern "C" rs_status rs_plan_inspect(const rs_key_desc *desc, uint64_t n, int with_values, rs_plan_info *out) {
  rs::g_last_error.clear();
  if (!desc || !out) return rs::fail(RS_ERR_NULL_ARG, "desc and out are required");
  rs::Plan p;
  std::string why;
  const bool pairs = with_values != 0;
  rs_status st = rs::make_plan(desc, n, pairs, rs::current_tuning(desc, n, pairs), &p, &why);
  if (st != RS_OK) return rs::fail(st, why);
  rs_plan_info r = {};
  r.form = p.local ? RS_FORM_LOCAL : p.literal ? RS_FORM_LITERAL : p.prescanned ? RS_FORM_PRESCANNED : RS_FORM_CHAINED;
  r.passes = p.literal ? 0 : p.npasses;
  r.tile_keys = p.tile;
  if (p.literal) {
    r.literal_cells = p.literal_cells;
    r.map_rows = p.map_rows;
    r.map_inner = p.map_inner;
    r.scan_chunk = rs::kBigScanChunk;
    r.off_counts = p.off_counts;
    r.off_map_lo = p.off_map_lo;
    r.off_map_hi = p.off_map_hi;
    r.off_starts = p.off_starts;
  }
  r.tmp_bytes = p.total;
  *out = r;
  return RS_OK;
}
