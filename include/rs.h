/*
 * rs.h -- C ABI of the MI355X (gfx950) Recombinant Sort library (librs.so).
 *
 * The method (Kumar, Gangal, Kumari, Tiwari, "Recombinant Sort: N-Dimensional
 * Cartesian Spaced Algorithm", arXiv 2107.01391):
 *   - every key is a fixed-width vector of N digits in base b, most
 *     significant first, zero padded (Section 3.1.2); decimals are stored as
 *     integers scaled by 10^lambda (Section 3.1, hashing cycle, and the
 *     n-digit version in the Supplementary section);
 *   - the hashing cycle counts the keys of every cell of the N-dimensional
 *     count space S (eq. (1), (2));
 *   - the extraction cycle walks the cells in lexicographic order and emits
 *     every cell's keys at a running output position (Section 3.2), which on
 *     the GPU is an exclusive scan of the counts followed by a stable scatter;
 *   - when b^N cells are too many for one space, the dimensions are split
 *     into groups sorted one after another (the bucket and radix parents of
 *     Sections 2.2 and 2.4).
 *
 * Conventions for every entry point:
 *   - Pointers named keys_* / vals_* / tmp / d_* are DEVICE pointers (memory
 *     from hipMalloc or a framework allocator on the current device).  The
 *     caller owns every buffer; the library allocates and frees nothing in
 *     the sort calls and keeps no pointer after the stream work completes.
 *   - Keys are aligned to their size (4 bytes for u32, 8 for u64 and fixed
 *     point, 16 for 16-byte strings), values to 4 bytes and tmp to 256
 *     bytes; anything else returns RS_ERR_UNSUPPORTED.  Arrays may start at
 *     any such element offset (slices of a larger buffer).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous: they enqueue kernels and return.  Errors found
 *     before launching are returned; faults during execution surface at the
 *     caller's next synchronisation.  Two exceptions wait on the stream:
 *     RS_FLAG_VALIDATE, and rs_sort_keys / rs_sort_pairs of base-27 strings
 *     of 16 symbols from 2^21 keys (the prescanned passes), which sort the
 *     buckets of the four leading symbols one by one and read back how many
 *     long buckets whose keys differ need the batched passes.  While the
 *     stream is being captured those strings run all eight passes instead,
 *     with no wait.
 *   - Order is ascending and stable: equal keys keep their input order
 *     (Section 1's definition of a stable sort; the position arithmetic of
 *     counting sort, Section 2.3).
 *   - keys_out may equal keys_in (and vals_out vals_in): the in-place
 *     overwrite of the extraction cycle (Section 3.2).  Other overlaps are
 *     undefined.
 *   - n == 0 is a no-op returning RS_OK.  Counts are 32-bit on the device:
 *     one array holds at most RS_MAX_ELEMENTS keys.
 *   - Keys must lie in the count space: 0 <= key < b^N for unsigned integers
 *     and fixed-point values, bytes in {0, 'a'..'z'} for base-27 strings
 *     (every value of the type for signed integers and base-256 strings,
 *     whose spaces cover the type).  With
 *     RS_FLAG_VALIDATE the library checks this first (a synchronous extra
 *     read) and returns RS_ERR_KEY_RANGE; without it, out-of-space keys give
 *     an unspecified order (never a fault).  8-byte keys of a space that
 *     fits 32 bits are carried as 32-bit words through large sorts, so an
 *     out-of-space one may also come back with only its low 32 bits.
 *   - No exception crosses the ABI and nothing aborts.  rs_last_error()
 *     returns a thread-local description of the last failure.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RS_MAX_ELEMENTS ((1ull << 30) - 1)

typedef enum rs_status {
  RS_OK = 0,
  RS_ERR_NULL_ARG = 1,      /* a required pointer is NULL */
  RS_ERR_BAD_DESC = 2,      /* key description inconsistent or unsupported values */
  RS_ERR_KEY_RANGE = 3,     /* RS_FLAG_VALIDATE found a key outside the count space */
  RS_ERR_TMP_TOO_SMALL = 4, /* tmp_bytes below what rs_*temp_bytes() asks for */
  RS_ERR_UNSUPPORTED = 5,   /* size or shape beyond the library's limits */
  RS_ERR_OOM = 6,           /* a host-side allocation failed (server only) */
  RS_ERR_HIP = 7,           /* a HIP runtime call or kernel launch failed */
  RS_ERR_BUSY = 8           /* server: no slot or memory for the request now */
} rs_status;

typedef enum rs_key_kind {
  RS_KEY_U32 = 0,       /* uint32_t keys */
  RS_KEY_U64 = 1,       /* uint64_t keys */
  RS_KEY_FIXED_I64 = 2, /* int64_t fixed-point: value * 10^frac_digits, >= 0 */
  RS_KEY_STR = 3,       /* fixed-width byte strings: base 27 (default), bytes in {0, 'a'..'z'};
                           base 256, any bytes (memcmp order) */
  RS_KEY_I32 = 4,       /* int32_t keys, full range: digits of key + 2^31 */
  RS_KEY_I64 = 5        /* int64_t keys, full range: digits of key + 2^63 */
} rs_key_kind;

#define RS_FLAG_VALIDATE 1u
/* Descending order, still stable (equal keys keep their input order): every
 * pass counts the complemented cell, cells - 1 - cell.  The paper's walk is
 * ascending; this is its mirror. */
#define RS_FLAG_DESCENDING 2u

/* Describes the key and its count space (Section 3.1.1: the digits of a key
 * are the coordinates of its cell). */
typedef struct rs_key_desc {
  uint32_t kind;        /* rs_key_kind */
  uint32_t base;        /* b, radix of one dimension; 0 = default: 256 for
                           U32/U64/I32/I64, 10 for FIXED_I64, 27 for STR
                           (pad + a..z; 256 = any byte) */
  uint32_t ndims;       /* N, digits per key; 0 = default: enough for the
                           type (4 / 8 base-256 digits, 19 base-10 digits,
                           str_width symbols) */
  uint32_t frac_digits; /* FIXED_I64: lambda, digits after the point; it
                           places the decimal point only and does not change
                           the order */
  uint32_t str_width;   /* STR: bytes per key (16 supported); N = str_width */
  uint32_t flags;       /* RS_FLAG_VALIDATE | RS_FLAG_DESCENDING */
} rs_key_desc;

/* Scratch bytes that rs_sort_keys (with_values = 0) or rs_sort_pairs
 * (with_values = 1) need for n keys of this description.  Writes *bytes.
 * Arrays of at most 4096 keys of 4 or 8 bytes are sorted whole in one
 * workgroup's LDS (every pass on chip, one launch); they need 256 bytes. */
rs_status rs_temp_bytes(const rs_key_desc *desc, uint64_t n, int with_values, size_t *bytes);

/* Sorts n keys.  Keys only: when the whole count space is small (b^N cells,
 * at most a few cells per key, and more than 4096 keys) this runs the
 * paper's literal form: count
 * every cell, scan the counts in lexicographic order, and write each cell's
 * count copies of the key rebuilt from the cell's coordinates (eq. (16));
 * otherwise it runs the grouped passes of rs_sort_pairs without payload.
 *   keys_in   [n] keys, layout by kind (strings: n rows of str_width bytes)
 *   keys_out  [n] sorted keys (may equal keys_in)
 *   tmp       scratch of at least rs_temp_bytes(desc, n, 0) bytes */
rs_status rs_sort_keys(const rs_key_desc *desc, const void *keys_in, void *keys_out, uint64_t n, void *tmp,
                       size_t tmp_bytes, void *stream);

/* Stable sort of n (key, uint32 value) pairs: for every group of digit
 * dimensions, least significant group first, one histogram of the group's
 * cells, an exclusive scan of the counts in lexicographic cell order, and a
 * stable scatter of keys and values to the scanned positions.
 *   vals_in   [n] uint32 payload
 *   vals_out  [n] payload permuted with the keys (may equal vals_in)
 *   tmp       scratch of at least rs_temp_bytes(desc, n, 1) bytes */
rs_status rs_sort_pairs(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                        uint32_t *vals_out, uint64_t n, void *tmp, size_t tmp_bytes, void *stream);

/* Size of the library's static device scratch (64 MiB per device). */
#define RS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* rs_sort_pairs without a tmp argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and rules as
 * rs_sort_pairs; the scratch is a static array inside the library, one
 * RS_NOALLOC_SCRATCH_BYTES copy per device, held from the first call on that
 * device until the process ends.  The call allocates nothing (no hipMalloc,
 * no hipFree).
 *   Limit: a sort whose rs_temp_bytes(desc, n, 1) exceeds
 *   RS_NOALLOC_SCRATCH_BYTES returns RS_ERR_UNSUPPORTED and launches nothing
 *   (with the default tuning: u32 pairs up to 8,134,272 keys, u64 pairs up
 *   to 5,478,208, 16-byte strings up to 2,360,192).
 *   Every call on a device shares that device's array: calls that overlap in
 *   time on one device (other streams or threads, no ordering between them)
 *   race and give unspecified results.  Calls ordered on one stream are safe;
 *   nothing a call leaves in the array affects the next one. */
rs_status rs_sort_pairs_noalloc(const rs_key_desc *desc, const void *keys_in, void *keys_out,
                                const uint32_t *vals_in, uint32_t *vals_out, uint64_t n, void *stream);

/* Scratch bytes for rs_sort_batched over nseg arrays holding `total` keys. */
rs_status rs_batched_temp_bytes(const rs_key_desc *desc, uint64_t total, uint32_t nseg, int with_values,
                                size_t *bytes);

/* Sorts nseg independent arrays in one launch sequence (bucket sort's
 * independent buckets, Section 2.2).  Array i is elements
 * [d_seg_offsets[i], d_seg_offsets[i+1]) of keys_in / vals_in and is written
 * to the same range of keys_out / vals_out, sorted on its own.
 *   d_seg_offsets  DEVICE array of nseg + 1 non-decreasing uint64 offsets,
 *                  d_seg_offsets[0] == 0 and d_seg_offsets[nseg] == total
 *   vals_in        NULL for keys only (then vals_out is ignored)
 * Arrays of at most a few thousand keys are sorted whole in on-chip memory
 * by one workgroup; larger ones run the grouped passes of rs_sort_pairs,
 * all arrays sharing every launch.  The launch shapes depend only on
 * (total, nseg), so a captured hipGraph can be replayed for any offsets with
 * the same (total, nseg).  Every array must hold at most RS_MAX_ELEMENTS
 * keys; total must be below 2^40.  Offsets that break these rules give an
 * unspecified order and unspecified contents of keys_out / vals_out, but no
 * access outside the buffers: every array's bounds are clamped to
 * [0, total) and RS_MAX_ELEMENTS keys on the device before use.  With
 * RS_FLAG_VALIDATE they are checked first and give RS_ERR_BAD_DESC. */
rs_status rs_sort_batched(const rs_key_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                          uint32_t *vals_out, const uint64_t *d_seg_offsets, uint32_t nseg, uint64_t total, void *tmp,
                          size_t tmp_bytes, void *stream);

/* Static description of a status code; never NULL. */
const char *rs_status_string(rs_status status);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *rs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
