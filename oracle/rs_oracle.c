/*
 * Recombinant Sort -- CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded implementation of the method of
 * "Recombinant Sort: N-Dimensional Cartesian Spaced Algorithm" (Kumar,
 * Gangal, Kumari, Tiwari; arXiv 2107.01391).  Only the test-suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes, step by step, in the paper's order:
 *
 *  1. Pre-processing (Section 3.1.2): every key is a fixed-width string of N
 *     digits in base b, most significant first, left-padded with zeros.
 *     Integers and fixed-point decimals (value * 10^lambda, already scaled
 *     when stored) give their base-b digits by division; a fixed-width
 *     string gives one digit per byte, 0 (pad) -> 0 and 'a'..'z' -> 1..26
 *     (base 27), or the byte itself (base 256: memcmp order of any bytes).
 *  2. Hashing cycle (Section 3.1, eq. (1), and the n-digit version in the
 *     Supplementary section): for every element, in input order, the cell
 *     S[d1][d2]..[dw] of the count space is incremented, and the traverse
 *     maps H_Min / H_Max are updated.
 *  3. Extraction cycle (Section 3.2 and Supplementary section): the cells are
 *     walked in lexicographic (raster) order, the first coordinate outermost,
 *     the inner coordinates bounded by the traverse maps; each occupied cell
 *     receives the running output position (the paper's overwrite position)
 *     and the position advances by the cell's count.  The walk stops when the
 *     position reaches the number of elements.  Every visited cell is counted
 *     into k, the extraction cost of Section 5.
 *  4. Emission: keys alone are written back as count copies of the value
 *     rebuilt from the cell's coordinates (eq. (16)); key/value pairs are
 *     placed by a second pass in input order, out[start[c]++] = element,
 *     which is counting sort's position arithmetic (Section 2.3) and keeps
 *     equal keys in input order.
 *  5. Hierarchy: when the N dimensions are too many for one count space they
 *     are split into consecutive groups (bucket sort's independent buckets,
 *     Section 2.2): each occupied cell of one level becomes a sub-array that
 *     is sorted by the next group.  Sub-arrays of one element stop early.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *  - Traverse maps in n dimensions: per value of the leading coordinate, one
 *    (touched flag, minimum) pair and one maximum for each inner coordinate,
 *    i.e. a per-row bounding box (sizes as in Table 3: 10x2 / 10x1 for two
 *    dimensions, 10x22 / 10x11 for three).  A one-dimensional space has a
 *    single (flag, minimum) and maximum.  Rows never touched are skipped.
 *  - The loop bound written "to H_Max+1" is exclusive, so the maximum itself
 *    is visited; "for z = 0 to S" emits exactly S copies.
 *  - Equal keys keep input order (stable), as the position arithmetic of
 *    counting sort gives.
 *  - Keys are non-negative; order is ascending.  Beyond the paper (which is
 *    silent on signs and on order): signed 32/64-bit integers are encoded
 *    by adding 2^31 / 2^63 (offset binary, which maps the signed order onto
 *    the unsigned one) before their digits are taken, and descending order
 *    walks the same cells in the mirrored raster order (every coordinate
 *    from its maximum down), with placement still in input order, so equal
 *    keys keep their input order in both directions.
 *
 * Parity of every function here is pinned by the CPU tests (worked example
 * of Section 3 / Example 1, Table 3's space shapes, brute-force stable sort
 * on small inputs, and the invariants of Section 4).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U32 = 0, ORC_U64 = 1, ORC_FIXED_I64 = 2, ORC_STR = 3, ORC_I32 = 4, ORC_I64 = 5 };
enum { ORC_ASCENDING = 0, ORC_DESCENDING = 1 };
enum {
  ORC_OK = 0,
  ORC_ERR_ARG = 1,      /* bad description / groups / pointers */
  ORC_ERR_KEY = 2,      /* a key outside [0, b^N) or outside the alphabet */
  ORC_ERR_SPACE = 3,    /* a count space larger than ORC_MAX_CELLS */
  ORC_ERR_MEM = 4,      /* allocation failed */
  ORC_ERR_INVARIANT = 5 /* a loop invariant of Section 4 did not hold */
};

#define ORC_MAX_DIMS 64
#define ORC_MAX_CELLS (1ull << 26)

typedef struct {
  uint32_t kind;      /* ORC_U32 / ORC_U64 / ORC_FIXED_I64 / ORC_STR / ORC_I32 / ORC_I64 */
  uint32_t base;      /* b: radix of every dimension */
  uint32_t ndims;     /* N: digits per key */
  uint32_t str_width; /* bytes per key for strings (= N) */
  uint32_t order;     /* ORC_ASCENDING or ORC_DESCENDING */
} orc_desc;

typedef struct {
  uint64_t cells_visited; /* k summed over every extraction cycle */
  uint64_t spaces;        /* number of count spaces built (hashing cycles) */
  uint64_t max_depth;     /* deepest hierarchy level used (1 = one level) */
} orc_stats;

/* ---------------------------------------------------------------- codec */

/* Strings over {pad, a..z} (base 27): pad -> 0, 'a'..'z' -> 1..26.  Strings
 * over every byte (base 256): the byte itself, which is memcmp order. */
static uint32_t str_symbol(uint32_t base, uint8_t byte) {
  if (base == 256) return byte;
  return byte == 0 ? 0u : (uint32_t)(byte - 'a') + 1u;
}
static uint8_t str_byte(uint32_t base, uint32_t sym) {
  if (base == 256) return (uint8_t)sym;
  return sym == 0 ? 0 : (uint8_t)('a' + sym - 1);
}

typedef struct {
  orc_desc d;
  const void *keys;
  uint64_t pw[ORC_MAX_DIMS + 1]; /* b^k, valid while it fits in 64 bits */
} codec;

/* The non-negative value whose base-b digits are the key's: the key itself,
 * or for signed integers the key plus 2^31 / 2^63. */
static uint64_t encoded(const codec *c, uint64_t i) {
  switch (c->d.kind) {
  case ORC_U32: return ((const uint32_t *)c->keys)[i];
  case ORC_I32: return (uint64_t)((int64_t)((const int32_t *)c->keys)[i] + 2147483648LL);
  case ORC_I64: return (uint64_t)((const int64_t *)c->keys)[i] ^ 0x8000000000000000ull;
  case ORC_FIXED_I64: return (uint64_t)((const int64_t *)c->keys)[i];
  default: return ((const uint64_t *)c->keys)[i];
  }
}

/* Digit j (0 = most significant) of element i: the paper's F_Numeric(t[j]). */
static uint32_t digit_of(const codec *c, uint64_t i, uint32_t j) {
  uint32_t n = c->d.ndims;
  switch (c->d.kind) {
  case ORC_I32:
  case ORC_I64:
    return (uint32_t)((encoded(c, i) / c->pw[n - 1 - j]) % c->d.base);
  case ORC_U32: {
    uint64_t v = ((const uint32_t *)c->keys)[i];
    return (uint32_t)((v / c->pw[n - 1 - j]) % c->d.base);
  }
  case ORC_U64: {
    uint64_t v = ((const uint64_t *)c->keys)[i];
    return (uint32_t)((v / c->pw[n - 1 - j]) % c->d.base);
  }
  case ORC_FIXED_I64: {
    uint64_t v = (uint64_t)((const int64_t *)c->keys)[i];
    return (uint32_t)((v / c->pw[n - 1 - j]) % c->d.base);
  }
  default: {
    const uint8_t *row = (const uint8_t *)c->keys + i * (uint64_t)c->d.str_width;
    return str_symbol(c->d.base, row[j]);
  }
  }
}

/* Checks the precondition of Section 3.1.2 on element i. */
static int key_valid(const codec *c, uint64_t i) {
  uint32_t n = c->d.ndims;
  if (c->d.kind == ORC_STR) {
    if (c->d.base == 256) return 1; /* every byte is a symbol */
    const uint8_t *row = (const uint8_t *)c->keys + i * (uint64_t)c->d.str_width;
    for (uint32_t j = 0; j < n; j++)
      if (row[j] != 0 && (row[j] < 'a' || row[j] > 'z')) return 0;
    return 1;
  }
  uint64_t v;
  if (c->d.kind == ORC_U32) v = ((const uint32_t *)c->keys)[i];
  else if (c->d.kind == ORC_U64) v = ((const uint64_t *)c->keys)[i];
  else if (c->d.kind == ORC_I32 || c->d.kind == ORC_I64) v = encoded(c, i);
  else {
    int64_t s = ((const int64_t *)c->keys)[i];
    if (s < 0) return 0;
    v = (uint64_t)s;
  }
  /* v < b^N, written without forming b^N when it overflows 64 bits */
  return (v / c->pw[n - 1]) < c->d.base;
}

static int codec_init(codec *c, const orc_desc *d, const void *keys) {
  if (!d || !keys) return ORC_ERR_ARG;
  if (d->ndims == 0 || d->ndims > ORC_MAX_DIMS || d->base < 2) return ORC_ERR_ARG;
  if (d->kind > ORC_I64 || d->order > ORC_DESCENDING) return ORC_ERR_ARG;
  if (d->kind == ORC_STR && ((d->base != 27 && d->base != 256) || d->str_width != d->ndims)) return ORC_ERR_ARG;
  c->d = *d;
  c->keys = keys;
  c->pw[0] = 1;
  for (uint32_t k = 1; k <= ORC_MAX_DIMS; k++) {
    if (c->pw[k - 1] > UINT64_MAX / d->base) { /* saturate: never divided by */
      for (; k <= ORC_MAX_DIMS; k++) c->pw[k] = UINT64_MAX;
      break;
    }
    c->pw[k] = c->pw[k - 1] * d->base;
  }
  if (d->kind != ORC_STR && c->pw[d->ndims - 1] == UINT64_MAX) return ORC_ERR_ARG;
  return ORC_OK;
}

/* ----------------------------------------------------- one count space */

/* The count space S of one level: w dimensions starting at dimension dlo,
 * b^w cells in row-major (lexicographic) order, plus its traverse maps. */
typedef struct {
  uint32_t dlo, w;
  uint64_t cells;
  uint64_t *S;         /* counts, kept all-zero between uses */
  uint64_t *start;     /* output position of each occupied cell */
  uint64_t *occupied;  /* occupied cells in walk order */
  uint64_t n_occupied;
  /* traverse maps: w == 1 -> a single entry; w >= 2 -> [b][w-1] */
  uint32_t *hmin_flag, *hmin, *hmax;
  uint64_t map_entries;
} space;

static int space_init(space *sp, const codec *c, uint32_t dlo, uint32_t w, uint64_t max_elems) {
  memset(sp, 0, sizeof *sp);
  sp->dlo = dlo;
  sp->w = w;
  if (w > 26) return ORC_ERR_SPACE;
  if (c->pw[w] == UINT64_MAX || c->pw[w] > ORC_MAX_CELLS) return ORC_ERR_SPACE;
  sp->cells = c->pw[w];
  sp->map_entries = (w == 1) ? 1 : (uint64_t)c->d.base * (w - 1);
  uint64_t occ = sp->cells < max_elems ? sp->cells : max_elems;
  if (occ == 0) occ = 1;
  sp->S = calloc(sp->cells, sizeof(uint64_t));
  sp->start = calloc(sp->cells, sizeof(uint64_t));
  sp->occupied = malloc(occ * sizeof(uint64_t));
  sp->hmin_flag = calloc(sp->map_entries, sizeof(uint32_t));
  sp->hmin = calloc(sp->map_entries, sizeof(uint32_t));
  sp->hmax = calloc(sp->map_entries, sizeof(uint32_t));
  if (!sp->S || !sp->start || !sp->occupied || !sp->hmin_flag || !sp->hmin || !sp->hmax)
    return ORC_ERR_MEM;
  return ORC_OK;
}

static void space_free(space *sp) {
  free(sp->S);
  free(sp->start);
  free(sp->occupied);
  free(sp->hmin_flag);
  free(sp->hmin);
  free(sp->hmax);
  memset(sp, 0, sizeof *sp);
}

/* Coordinates (d1..dw) of element i in this space, and its row-major cell. */
static uint64_t element_cell(const codec *c, const space *sp, uint64_t i, uint32_t *coord) {
  uint64_t cell = 0;
  for (uint32_t t = 0; t < sp->w; t++) {
    coord[t] = digit_of(c, i, sp->dlo + t);
    cell = cell * c->d.base + coord[t];
  }
  return cell;
}

/* Traverse-map update for one element (the H_Max / H_Min steps of the
 * hashing cycle): per leading coordinate, the smallest and largest value
 * seen in each inner coordinate; for one dimension, of the single one. */
static void maps_update(space *sp, uint32_t base, const uint32_t *coord) {
  if (sp->w == 1) {
    if (sp->hmax[0] < coord[0]) sp->hmax[0] = coord[0];
    if (sp->hmin_flag[0] == 0) {
      sp->hmin[0] = coord[0];
      sp->hmin_flag[0] = 1;
    } else if (sp->hmin[0] > coord[0]) {
      sp->hmin[0] = coord[0];
    }
    return;
  }
  (void)base;
  uint64_t row = (uint64_t)coord[0] * (sp->w - 1);
  for (uint32_t j = 1; j < sp->w; j++) {
    uint64_t e = row + (j - 1);
    if (sp->hmax[e] < coord[j]) sp->hmax[e] = coord[j];
    if (sp->hmin_flag[e] == 0) {
      sp->hmin[e] = coord[j];
      sp->hmin_flag[e] = 1;
    } else if (sp->hmin[e] > coord[j]) {
      sp->hmin[e] = coord[j];
    }
  }
}

/* Hashing cycle over the elements items[0..cnt): S[cell]++ (eq. (1)). */
static void hashing_cycle(const codec *c, space *sp, const uint64_t *items, uint64_t cnt) {
  uint32_t coord[ORC_MAX_DIMS];
  memset(sp->hmin_flag, 0, sp->map_entries * sizeof(uint32_t));
  memset(sp->hmin, 0, sp->map_entries * sizeof(uint32_t));
  memset(sp->hmax, 0, sp->map_entries * sizeof(uint32_t));
  for (uint64_t i = 0; i < cnt; i++) {
    uint64_t cell = element_cell(c, sp, items[i], coord);
    sp->S[cell] += 1;
    maps_update(sp, c->d.base, coord);
  }
}

/* Visits one cell of the extraction walk; returns 1 when every element has
 * been given a position (the early return of the extraction cycle). */
static int visit(space *sp, uint64_t cell, uint64_t *pos, uint64_t cnt, uint64_t *k) {
  *k += 1;
  if (sp->S[cell] != 0) {
    sp->start[cell] = *pos;
    sp->occupied[sp->n_occupied++] = cell;
    *pos += sp->S[cell];
  }
  return *pos == cnt;
}

/* Extraction cycle: raster walk of the space in lexicographic order, bounded
 * by the traverse maps.  Returns the number of positions handed out. */
static uint64_t extraction_walk(const codec *c, space *sp, uint64_t cnt, uint64_t *k) {
  uint64_t pos = 0;
  uint32_t b = c->d.base;
  sp->n_occupied = 0;
  if (cnt == 0) return 0;
  const int down = c->d.order == ORC_DESCENDING;
  if (sp->w == 1) {
    if (!sp->hmin_flag[0]) return 0;
    for (uint64_t t = 0; t <= sp->hmax[0] - sp->hmin[0]; t++) {
      const uint64_t x = down ? sp->hmax[0] - t : sp->hmin[0] + t;
      if (visit(sp, x, &pos, cnt, k)) return pos;
    }
    return pos;
  }
  /* ascending: every coordinate from its minimum up; descending: the same
   * bounds walked from the maximum down (the mirrored raster order) */
  uint32_t lo[ORC_MAX_DIMS], hi[ORC_MAX_DIMS], cur[ORC_MAX_DIMS];
  for (uint32_t t = 0; t < b; t++) {
    const uint32_t r = down ? b - 1 - t : t;
    uint64_t row = (uint64_t)r * (sp->w - 1);
    if (!sp->hmin_flag[row]) continue; /* row never touched */
    for (uint32_t j = 1; j < sp->w; j++) {
      lo[j] = sp->hmin[row + j - 1];
      hi[j] = sp->hmax[row + j - 1];
      cur[j] = down ? hi[j] : lo[j];
    }
    for (;;) {
      uint64_t cell = r;
      for (uint32_t j = 1; j < sp->w; j++) cell = cell * b + cur[j];
      if (visit(sp, cell, &pos, cnt, k)) return pos;
      /* next coordinate vector: the last dimension counts fastest */
      int32_t j = (int32_t)sp->w - 1;
      while (j >= 1) {
        if (!down && cur[j] < hi[j]) {
          cur[j]++;
          break;
        }
        if (down && cur[j] > lo[j]) {
          cur[j]--;
          break;
        }
        cur[j] = down ? hi[j] : lo[j];
        j--;
      }
      if (j == 0) break;
    }
  }
  return pos;
}

/* --------------------------------------------------------- the hierarchy */

typedef struct {
  codec c;
  void *keys_out;
  const uint32_t *vals_in; /* NULL: keys only */
  uint32_t ngroups;
  space sp[ORC_MAX_DIMS];
  uint64_t *tmp;           /* placement buffer, n entries */
  uint32_t prefix_sym[ORC_MAX_DIMS];
  orc_stats st;
} sorter;

static void write_rebuilt(sorter *s, uint64_t pos, uint64_t prefix, const space *sp, uint64_t cell) {
  const codec *c = &s->c;
  if (c->d.kind == ORC_STR) {
    uint8_t *row = (uint8_t *)s->keys_out + pos * (uint64_t)c->d.str_width;
    for (uint32_t j = 0; j < sp->dlo; j++) row[j] = str_byte(c->d.base, s->prefix_sym[j]);
    uint64_t rest = cell;
    for (int32_t t = (int32_t)sp->w - 1; t >= 0; t--) {
      row[sp->dlo + t] = str_byte(c->d.base, (uint32_t)(rest % c->d.base));
      rest /= c->d.base;
    }
    return;
  }
  /* eq. (16): the element is its coordinates read as one base-b numeral
   * (signed keys: minus the bias their digits were taken with) */
  uint64_t v = prefix * c->pw[sp->w] + cell;
  if (c->d.kind == ORC_U32) ((uint32_t *)s->keys_out)[pos] = (uint32_t)v;
  else if (c->d.kind == ORC_U64) ((uint64_t *)s->keys_out)[pos] = v;
  else if (c->d.kind == ORC_I32) ((int32_t *)s->keys_out)[pos] = (int32_t)((int64_t)v - 2147483648LL);
  else if (c->d.kind == ORC_I64) ((uint64_t *)s->keys_out)[pos] = v ^ 0x8000000000000000ull;
  else ((int64_t *)s->keys_out)[pos] = (int64_t)v;
}

static void copy_key(sorter *s, uint64_t pos, uint64_t elem) {
  const codec *c = &s->c;
  if (c->d.kind == ORC_STR) {
    memcpy((uint8_t *)s->keys_out + pos * (uint64_t)c->d.str_width,
           (const uint8_t *)c->keys + elem * (uint64_t)c->d.str_width, c->d.str_width);
  } else if (c->d.kind == ORC_U32 || c->d.kind == ORC_I32) {
    ((uint32_t *)s->keys_out)[pos] = ((const uint32_t *)c->keys)[elem];
  } else {
    ((uint64_t *)s->keys_out)[pos] = ((const uint64_t *)c->keys)[elem];
  }
}

/* Sorts the sub-array items[0..cnt) (already ordered by every earlier level)
 * by dimension group g.  base = its offset in the output, prefix = the value
 * of the coordinates fixed by earlier levels. */
static int sort_level(sorter *s, uint64_t *items, uint64_t cnt, uint32_t g, uint64_t base, uint64_t prefix) {
  const codec *c = &s->c;
  space *sp = &s->sp[g];
  int leaf = (g + 1 == s->ngroups);
  if (g + 1 > s->st.max_depth) s->st.max_depth = g + 1;
  s->st.spaces += 1;

  hashing_cycle(c, sp, items, cnt);
  uint64_t k = 0;
  uint64_t placed = extraction_walk(c, sp, cnt, &k);
  s->st.cells_visited += k;

  /* I_Hash at termination (Section 4.1): every element was mapped, so the
   * counts of the occupied cells add up to the number of elements. */
  uint64_t total = 0;
  for (uint64_t o = 0; o < sp->n_occupied; o++) total += sp->S[sp->occupied[o]];
  if (total != cnt || placed != cnt) return ORC_ERR_INVARIANT;

  uint32_t coord[ORC_MAX_DIMS];
  if (leaf && s->vals_in == NULL) {
    /* keys only, all dimensions fixed: S[c] copies of the rebuilt element */
    for (uint64_t o = 0; o < sp->n_occupied; o++) {
      uint64_t cell = sp->occupied[o];
      for (uint64_t z = 0; z < sp->S[cell]; z++) write_rebuilt(s, base + sp->start[cell] + z, prefix, sp, cell);
    }
  } else {
    /* stable placement in input order: out[start[c]++] = element */
    for (uint64_t i = 0; i < cnt; i++) {
      uint64_t cell = element_cell(c, sp, items[i], coord);
      s->tmp[sp->start[cell]++] = items[i];
    }
    memcpy(items, s->tmp, cnt * sizeof(uint64_t));
    for (uint64_t o = 0; o < sp->n_occupied; o++) {
      uint64_t cell = sp->occupied[o];
      sp->start[cell] -= sp->S[cell];
    }
  }

  if (!leaf) {
    /* the occupied list and counts of this level are consumed before the
     * space is reused by a sibling, so copy what the recursion needs */
    uint64_t nocc = sp->n_occupied;
    uint64_t *cells = malloc((nocc ? nocc : 1) * 3 * sizeof(uint64_t));
    if (!cells) return ORC_ERR_MEM;
    for (uint64_t o = 0; o < nocc; o++) {
      uint64_t cell = sp->occupied[o];
      cells[3 * o] = cell;
      cells[3 * o + 1] = sp->start[cell];
      cells[3 * o + 2] = sp->S[cell];
      sp->S[cell] = 0;
    }
    int rc = ORC_OK;
    for (uint64_t o = 0; o < nocc && rc == ORC_OK; o++) {
      uint64_t cell = cells[3 * o], st = cells[3 * o + 1], m = cells[3 * o + 2];
      if (m == 1) {
        if (s->vals_in == NULL) copy_key(s, base + st, items[st]);
        continue;
      }
      if (c->d.kind == ORC_STR) {
        uint64_t rest = cell;
        for (int32_t t = (int32_t)sp->w - 1; t >= 0; t--) {
          s->prefix_sym[sp->dlo + t] = (uint32_t)(rest % c->d.base);
          rest /= c->d.base;
        }
      }
      rc = sort_level(s, items + st, m, g + 1, base + st, prefix * c->pw[sp->w] + cell);
    }
    free(cells);
    return rc;
  }
  for (uint64_t o = 0; o < sp->n_occupied; o++) sp->S[sp->occupied[o]] = 0;
  return ORC_OK;
}

static void sorter_free(sorter *s) {
  for (uint32_t g = 0; g < s->ngroups; g++) space_free(&s->sp[g]);
  free(s->tmp);
}

/* Sorts n keys (and their uint32 payload when vals_in is not NULL) in
 * desc->order, stable.  groups[0..ngroups) are the widths of the dimension groups of
 * the hierarchy, most significant first; they must add up to N. */
int orc_sort(const orc_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
             uint32_t *vals_out, uint64_t n, const uint32_t *groups, uint32_t ngroups, orc_stats *stats) {
  sorter *s = calloc(1, sizeof(sorter));
  if (!s) return ORC_ERR_MEM;
  int rc = codec_init(&s->c, desc, keys_in);
  if (rc == ORC_OK && (!keys_out || !groups || ngroups == 0 || ngroups > ORC_MAX_DIMS)) rc = ORC_ERR_ARG;
  if (rc == ORC_OK && vals_in && !vals_out) rc = ORC_ERR_ARG;
  if (rc == ORC_OK) {
    uint32_t sum = 0;
    for (uint32_t g = 0; g < ngroups; g++) {
      if (groups[g] == 0) rc = ORC_ERR_ARG;
      sum += groups[g];
    }
    if (sum != desc->ndims) rc = ORC_ERR_ARG;
  }
  for (uint64_t i = 0; rc == ORC_OK && i < n; i++)
    if (!key_valid(&s->c, i)) rc = ORC_ERR_KEY;
  if (rc != ORC_OK) {
    free(s);
    return rc;
  }
  s->keys_out = keys_out;
  s->vals_in = vals_in;
  s->ngroups = ngroups;
  uint32_t dlo = 0;
  for (uint32_t g = 0; g < ngroups && rc == ORC_OK; g++) {
    rc = space_init(&s->sp[g], &s->c, dlo, groups[g], n);
    dlo += groups[g];
  }
  uint64_t *items = malloc((n ? n : 1) * sizeof(uint64_t));
  s->tmp = malloc((n ? n : 1) * sizeof(uint64_t));
  if (rc == ORC_OK && (!items || !s->tmp)) rc = ORC_ERR_MEM;
  if (rc == ORC_OK) {
    for (uint64_t i = 0; i < n; i++) items[i] = i;
    if (n == 1) {
      copy_key(s, 0, 0);
    } else if (n > 1) {
      rc = sort_level(s, items, n, 0, 0, 0);
    }
  }
  if (rc == ORC_OK && vals_in) {
    for (uint64_t i = 0; i < n; i++) {
      copy_key(s, i, items[i]);
      vals_out[i] = vals_in[items[i]];
    }
  }
  if (stats) *stats = s->st;
  free(items);
  sorter_free(s);
  free(s);
  return rc;
}

/* Sorts nseg independent arrays: segment i is [offsets[i], offsets[i+1]) of
 * the inputs; each is sorted on its own with the same hierarchy. */
int orc_sort_segments(const orc_desc *desc, const void *keys_in, void *keys_out, const uint32_t *vals_in,
                      uint32_t *vals_out, const uint64_t *offsets, uint32_t nseg, const uint32_t *groups,
                      uint32_t ngroups, orc_stats *stats) {
  orc_stats total = {0, 0, 0};
  uint64_t width = desc->kind == ORC_STR ? desc->str_width : (desc->kind == ORC_U32 || desc->kind == ORC_I32 ? 4 : 8);
  for (uint32_t i = 0; i < nseg; i++) {
    uint64_t a = offsets[i], b = offsets[i + 1];
    if (b < a) return ORC_ERR_ARG;
    orc_stats st;
    int rc = orc_sort(desc, (const uint8_t *)keys_in + a * width, (uint8_t *)keys_out + a * width,
                      vals_in ? vals_in + a : NULL, vals_out ? vals_out + a : NULL, b - a, groups, ngroups, &st);
    if (rc != ORC_OK) return rc;
    total.cells_visited += st.cells_visited;
    total.spaces += st.spaces;
    if (st.max_depth > total.max_depth) total.max_depth = st.max_depth;
  }
  if (stats) *stats = total;
  return ORC_OK;
}

/* One level over the whole input, exposed for inspection: the hashing cycle
 * (counts S[b^w] and traverse maps) and the extraction walk (start positions
 * S-occupied cells, cost k).  Map arrays hold map_entries values: 1 for a
 * one-dimensional space, b*(w-1) otherwise ([row][inner dimension]). */
int orc_hash_level(const orc_desc *desc, const void *keys, uint64_t n, uint32_t dlo, uint32_t w, uint64_t *S_out,
                   uint64_t *start_out, uint32_t *hmin_flag_out, uint32_t *hmin_out, uint32_t *hmax_out,
                   uint64_t *k_out) {
  codec c;
  int rc = codec_init(&c, desc, keys);
  if (rc != ORC_OK) return rc;
  if (w == 0 || dlo + w > desc->ndims) return ORC_ERR_ARG;
  for (uint64_t i = 0; i < n; i++)
    if (!key_valid(&c, i)) return ORC_ERR_KEY;
  space sp;
  rc = space_init(&sp, &c, dlo, w, n);
  if (rc != ORC_OK) {
    space_free(&sp);
    return rc;
  }
  uint64_t *items = malloc((n ? n : 1) * sizeof(uint64_t));
  if (!items) {
    space_free(&sp);
    return ORC_ERR_MEM;
  }
  for (uint64_t i = 0; i < n; i++) items[i] = i;
  hashing_cycle(&c, &sp, items, n);
  uint64_t k = 0;
  extraction_walk(&c, &sp, n, &k);
  memcpy(S_out, sp.S, sp.cells * sizeof(uint64_t));
  memset(start_out, 0, sp.cells * sizeof(uint64_t));
  for (uint64_t o = 0; o < sp.n_occupied; o++) start_out[sp.occupied[o]] = sp.start[sp.occupied[o]];
  memcpy(hmin_flag_out, sp.hmin_flag, sp.map_entries * sizeof(uint32_t));
  memcpy(hmin_out, sp.hmin, sp.map_entries * sizeof(uint32_t));
  memcpy(hmax_out, sp.hmax, sp.map_entries * sizeof(uint32_t));
  *k_out = k;
  free(items);
  space_free(&sp);
  return ORC_OK;
}

/* Number of base-b digits needed for every value below max_exclusive
 * (Table 3: the dimensions of the count space for a data range). */
uint32_t orc_dims_for(uint64_t max_exclusive, uint32_t base) {
  uint64_t top = max_exclusive ? max_exclusive - 1 : 0;
  uint32_t d = 1;
  while (top >= base) {
    top /= base;
    d++;
  }
  return d;
}
