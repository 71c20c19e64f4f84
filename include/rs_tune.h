/*
 * rs_tune.h -- the autotuner of librs.so.
 *
 * The paper leaves free how the N digit dimensions are grouped into count
 * spaces (the hierarchy of Section 2.2: one count space per group), and
 * every grouping gives the same sorted output.  On the GPU the grouping,
 * together with the tile shape of the kernels, decides the speed.  The
 * tuner times the candidate choices on the caller's own data and stream
 * and keeps the fastest per (key description, payload or not, single or
 * batched, size class = floor(log2 n)).  Later sorts of the same class use
 * the kept choice.  Results never depend on the choice.
 *
 * Precedence of the choice a sort uses: the environment variables
 * RS_DIGIT_BITS, RS_MAX_CELLS, RS_TILE_BLOCK, RS_PRESCAN_MIN_N (testing),
 * then the tuned choice of the size class, then the defaults.
 *
 * The tuning table is process-wide and protected by a lock.  Tuning itself
 * runs sorts on the given stream and synchronizes it.
 */
#ifndef RS_TUNE_H
#define RS_TUNE_H

#include <stddef.h>
#include <stdint.h>

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_tuning {
  uint32_t digit_bits;    /* bits per pass for power-of-two bases (4..11) */
  uint32_t max_cells;     /* largest count space of one pass for other bases (2..2048) */
  uint32_t tile_block;    /* threads per tile of prescanned passes: 256 or 512 */
  uint32_t reserved;      /* 0 */
  uint64_t prescan_min_n; /* single arrays from this length use prescanned passes */
} rs_tuning;

/* The choice a sort of n keys would use now.  batched != 0: the batched
 * form over n keys in all. */
rs_status rs_tuning_get(const rs_key_desc *desc, uint64_t n, int with_values, int batched, rs_tuning *out);

/* Keeps `t` for the size class of n (replacing a tuned choice).  Fields out
 * of range give RS_ERR_BAD_DESC. */
rs_status rs_tuning_set(const rs_key_desc *desc, uint64_t n, int with_values, int batched, const rs_tuning *t);

/* Forgets every kept choice. */
rs_status rs_tuning_clear(void);

/* Scratch for rs_tune_sort / rs_tune_batched: the largest tmp any candidate
 * needs (nseg = 0: single array of n keys; else the batched form over nseg
 * arrays holding n keys). */
rs_status rs_tune_temp_bytes(const rs_key_desc *desc, uint64_t n, uint32_t nseg, int with_values, size_t *bytes);

/* Times every candidate on keys_in / vals_in (vals_in NULL: keys only),
 * sorting into keys_out / vals_out (n elements each, distinct from the
 * inputs, which are left unchanged), `reps` timed runs after one warm-up
 * (0 = 3), and keeps the fastest for the size class of n.  best / best_ms
 * (either may be NULL) receive the kept choice and its mean time.
 * Synchronous: returns after the stream's work is done. */
rs_status rs_tune_sort(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                       uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream, uint32_t reps,
                       rs_tuning *best, double *best_ms);

/* The same for the batched form over nseg arrays (d_seg_offsets as for
 * rs_sort_batched). */
rs_status rs_tune_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                          uint32_t *vals_out, const uint64_t *d_seg_offsets, uint32_t nseg, uint64_t total, void *tmp,
                          size_t tmp_bytes, void *stream, uint32_t reps, rs_tuning *best, double *best_ms);

/* Writes / reads the kept choices as text, one per line.  Loading adds to
 * (and overrides) the table. */
rs_status rs_tuning_save(const char *path);
rs_status rs_tuning_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* RS_TUNE_H */
