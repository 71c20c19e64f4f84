/*
 * rs_inspect.h -- what a sort of librs.so will do, without running it.
 *
 * The planner picks one of four forms for a single array (see rs.h):
 *   RS_FORM_LOCAL       at most 4096 keys of 4 or 8 bytes: one workgroup
 *                       sorts the array whole in on-chip memory;
 *   RS_FORM_LITERAL     keys only on a small integer space: the paper's own
 *                       extraction -- count every cell of the whole space
 *                       (the hashing cycle, eq. (1)), walk the cells in
 *                       lexicographic order (Section 3.2), write each
 *                       cell's count copies of its rebuilt key (eq. (16));
 *                       the count kernel keeps the traverse maps (Section
 *                       3.1: per value of the leading coordinate, the
 *                       occupied range of the row), and the walk skips the
 *                       4096-cell chunks that no row's range reaches;
 *   RS_FORM_CHAINED     grouped passes, tiles chained by look-back;
 *   RS_FORM_PRESCANNED  grouped passes, per-tile counts and one scan.
 * For the literal form the scratch layout is reported too, so that a caller
 * (or a test) can read the counts, the maps and the starts back from tmp
 * after the sort.
 */
#ifndef RS_INSPECT_H
#define RS_INSPECT_H

#include <stddef.h>
#include <stdint.h>

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RS_FORM_LOCAL 0u
#define RS_FORM_LITERAL 1u
#define RS_FORM_CHAINED 2u
#define RS_FORM_PRESCANNED 3u

typedef struct rs_plan_info {
  uint32_t form;          /* RS_FORM_* */
  uint32_t passes;        /* grouped passes (0 for the literal form) */
  uint32_t tile_keys;     /* keys per tile of the passes */
  uint32_t literal_cells; /* literal form: cells of the whole space, b^N */
  uint32_t map_rows;      /* literal form: traverse-map rows, one per value of the leading coordinate */
  uint32_t map_inner;     /* literal form: cells per row, b^(N-1) (b^N for one dimension) */
  uint32_t scan_chunk;    /* literal form: cells per chunk of the walk (a skipped chunk is not read) */
  uint32_t reserved;
  /* literal form: byte offsets into tmp, each an array of uint32 --
   *   off_counts  [literal_cells] count of every cell (row-major)
   *   off_map_lo  [map_rows] complemented least occupied offset in the row
   *               (~lo; 0 = row never touched)
   *   off_map_hi  [map_rows] greatest occupied offset in the row
   *   off_starts  [literal_cells] output position of every cell, written
   *               only in chunks that some row's occupied range reaches */
  uint64_t off_counts, off_map_lo, off_map_hi, off_starts;
  uint64_t tmp_bytes;     /* what rs_temp_bytes reports */
} rs_plan_info;

/* The plan rs_sort_keys (with_values = 0) or rs_sort_pairs (with_values = 1)
 * would use for n keys of this description with the current tuning.
 * Host only: nothing is launched. */
rs_status rs_plan_inspect(const rs_key_desc *desc, uint64_t n, int with_values, rs_plan_info *out);

#ifdef __cplusplus
}
#endif

#endif /* RS_INSPECT_H */
