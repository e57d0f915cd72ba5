/*
 * CPU oracle for the columnar query hot path. TEST INFRASTRUCTURE ONLY:
 * it is called by the test suite, by the smoke check and by the CPU-baseline
 * leg of the benchmark, never by the product path. It shares no source with
 * the GPU library.
 *
 * The paper hands its operators (scans, filters, joins, aggregations) to a
 * GPU library and defines no semantics of its own for them (Section 2,
 * Background). Every step of the hot path therefore reaches exactly the result
 * of the plain relational definition over multisets of rows, and this file
 * writes that definition out:
 *
 *   selection   a row passes iff lo_j <= col_j <= hi_j for every predicate j
 *   projection  e(r) = prod_f (sign_f * col_f[r] + add_f), two's-complement
 *               arithmetic modulo 2^64, evaluated left to right
 *   group-by    sort the passing rows by key, one output row per run:
 *               COUNT, SUM_j (mod 2^64), AVG_j = (double)SUM_j / (double)COUNT
 *   equi-join   sort both sides by key, every (probe, build) pair with equal
 *               keys (inner join), reported in (probe_row, build_row) order
 *   partition   p(k) = (k * 0x9E3779B97F4A7C15 mod 2^64) >> (64 - b).
 *               Section 3.2 (Example Execution) hash-partitions both sides
 *               of a join but names no hash function; this 64-bit
 *               multiplicative hash with Knuth's constant (floor(2^64 /
 *               golden ratio)) is the workload's choice. A stable counting
 *               sort yields the partitions in row order
 *
 * Values are widened to int64 before any comparison: uint8 by zero extension,
 * int32 by sign extension. An __int128 shadow of every product and sum flags
 * results whose exact value leaves the int64 range; the flag is reported and
 * never changes a result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  const void* data;
  int32_t width; /* 1 = uint8, 4 = int32, 8 = int64 */
} oc_col;

static int64_t widen(const oc_col* c, int64_t r) {
  switch (c->width) {
    case 1: return (int64_t)((const uint8_t*)c->data)[r];
    case 4: return (int64_t)((const int32_t*)c->data)[r];
    default: return ((const int64_t*)c->data)[r];
  }
}

static int fits_i64(__int128 v) { return v >= (__int128)INT64_MIN && v <= (__int128)INT64_MAX; }

/* Selection (sigma): conjunction of inclusive ranges. Returns the pass count. */
int64_t oc_filter(const oc_col* cols, int64_t n, int32_t np, const int32_t* pcol, const int64_t* plo,
                  const int64_t* phi, uint8_t* pass) {
  int64_t count = 0;
  for (int64_t r = 0; r < n; r++) {
    int ok = 1;
    for (int32_t j = 0; j < np && ok; j++) {
      int64_t v = widen(&cols[pcol[j]], r);
      if (v < plo[j] || v > phi[j]) ok = 0;
    }
    pass[r] = (uint8_t)ok;
    count += ok;
  }
  return count;
}

/* Projection (pi) of one product expression. fcol[f] < 0 means the constant
 * fadd[f]. out[r] is the wrapped int64 value; ovf[r] (nullable) is set when an
 * intermediate exact value leaves the int64 range. */
void oc_project(const oc_col* cols, int64_t n, int32_t nf, const int32_t* fcol, const int64_t* fsign,
                const int64_t* fadd, int64_t* out, uint8_t* ovf) {
  for (int64_t r = 0; r < n; r++) {
    uint64_t acc = 1;
    int flag = 0;
    for (int32_t f = 0; f < nf; f++) {
      int64_t x = fcol[f] < 0 ? 0 : widen(&cols[fcol[f]], r);
      __int128 exact_factor = (__int128)fsign[f] * x + fadd[f];
      uint64_t factor = (uint64_t)fsign[f] * (uint64_t)x + (uint64_t)fadd[f];
      if (!fits_i64(exact_factor)) flag = 1;
      __int128 exact_prod = (__int128)(int64_t)acc * (__int128)(int64_t)factor;
      if (f > 0 && !fits_i64(exact_prod)) flag = 1;
      acc = (f == 0) ? factor : acc * factor;
    }
    out[r] = (int64_t)acc;
    if (ovf) ovf[r] = (uint8_t)flag;
  }
}

/* ---- group-by ------------------------------------------------------------ */

typedef struct {
  int64_t k0, k1;
  int64_t row;
} keyed_row;

static int cmp_keyed_row(const void* a, const void* b) {
  const keyed_row* x = (const keyed_row*)a;
  const keyed_row* y = (const keyed_row*)b;
  if (x->k0 != y->k0) return x->k0 < y->k0 ? -1 : 1;
  if (x->k1 != y->k1) return x->k1 < y->k1 ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

/* Group-by (gamma) with COUNT, SUM and AVG over nval int64 value arrays.
 * Groups are the distinct key tuples (1 or 2 key columns) of passing rows,
 * emitted in ascending lexicographic key order. Returns the group count, or
 * -1 if it exceeds max_groups. out_keys is [g][nkey]; out_sums, out_avg and
 * out_ovf are [g][nval]. */
int64_t oc_groupby(int64_t n, const uint8_t* pass, int32_t nkey, const oc_col* keys, int32_t nval,
                   const int64_t* const* vals, int64_t* out_keys, int64_t* out_count, int64_t* out_sums,
                   double* out_avg, uint8_t* out_ovf, int64_t max_groups) {
  int64_t m = 0;
  for (int64_t r = 0; r < n; r++) m += (pass == NULL || pass[r]);
  keyed_row* rows = (keyed_row*)malloc((size_t)(m > 0 ? m : 1) * sizeof(keyed_row));
  int64_t w = 0;
  for (int64_t r = 0; r < n; r++) {
    if (pass != NULL && !pass[r]) continue;
    rows[w].k0 = widen(&keys[0], r);
    rows[w].k1 = nkey > 1 ? widen(&keys[1], r) : 0;
    rows[w].row = r;
    w++;
  }
  qsort(rows, (size_t)m, sizeof(keyed_row), cmp_keyed_row);

  int64_t g = 0;
  for (int64_t i = 0; i < m;) {
    int64_t j = i;
    while (j < m && rows[j].k0 == rows[i].k0 && rows[j].k1 == rows[i].k1) j++;
    if (g >= max_groups) {
      free(rows);
      return -1;
    }
    out_keys[g * nkey + 0] = rows[i].k0;
    if (nkey > 1) out_keys[g * nkey + 1] = rows[i].k1;
    int64_t count = j - i;
    out_count[g] = count;
    for (int32_t v = 0; v < nval; v++) {
      uint64_t s = 0;
      __int128 exact = 0;
      int flag = 0;
      for (int64_t t = i; t < j; t++) {
        int64_t x = vals[v][rows[t].row];
        s += (uint64_t)x;
        exact += x;
        if (!fits_i64(exact)) flag = 1;
      }
      out_sums[g * nval + v] = (int64_t)s;
      out_avg[g * nval + v] = (double)(int64_t)s / (double)count;
      if (out_ovf) out_ovf[g * nval + v] = (uint8_t)flag;
    }
    g++;
    i = j;
  }
  free(rows);
  return g;
}

/* ---- equi-join ----------------------------------------------------------- */

typedef struct {
  int64_t key, row;
} key_row;

static int cmp_key_row(const void* a, const void* b) {
  const key_row* x = (const key_row*)a;
  const key_row* y = (const key_row*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

typedef struct {
  int64_t probe, build;
} pair_rows;

static int cmp_pair(const void* a, const void* b) {
  const pair_rows* x = (const pair_rows*)a;
  const pair_rows* y = (const pair_rows*)b;
  if (x->probe != y->probe) return x->probe < y->probe ? -1 : 1;
  if (x->build != y->build) return x->build < y->build ? -1 : 1;
  return 0;
}

static key_row* sorted_side(const int64_t* keys, int64_t n, const uint8_t* pass, int64_t* m_out) {
  int64_t m = 0;
  for (int64_t r = 0; r < n; r++) m += (pass == NULL || pass[r]);
  key_row* v = (key_row*)malloc((size_t)(m > 0 ? m : 1) * sizeof(key_row));
  int64_t w = 0;
  for (int64_t r = 0; r < n; r++)
    if (pass == NULL || pass[r]) {
      v[w].key = keys[r];
      v[w].row = r;
      w++;
    }
  qsort(v, (size_t)m, sizeof(key_row), cmp_key_row);
  *m_out = m;
  return v;
}

/* Inner equi-join of the passing build rows with the passing probe rows.
 * Returns the exact cardinality; writes min(cardinality, cap) pairs ordered by
 * (probe_row, build_row). Output arrays may be NULL when cap == 0. */
int64_t oc_join(const int64_t* bkeys, int64_t nb, const uint8_t* bpass, const int64_t* pkeys, int64_t np,
                const uint8_t* ppass, int64_t* out_probe, int64_t* out_build, int64_t cap) {
  int64_t mb, mp;
  key_row* B = sorted_side(bkeys, nb, bpass, &mb);
  key_row* P = sorted_side(pkeys, np, ppass, &mp);
  int64_t total = 0;
  for (int64_t i = 0, j = 0; i < mb && j < mp;) {
    if (B[i].key < P[j].key) { i++; continue; }
    if (B[i].key > P[j].key) { j++; continue; }
    int64_t i2 = i, j2 = j;
    while (i2 < mb && B[i2].key == B[i].key) i2++;
    while (j2 < mp && P[j2].key == P[j].key) j2++;
    total += (i2 - i) * (j2 - j);
    i = i2;
    j = j2;
  }
  if (cap > 0 && total > 0) {
    int64_t keep = total < cap ? total : cap;
    pair_rows* out = (pair_rows*)malloc((size_t)total * sizeof(pair_rows));
    int64_t w = 0;
    for (int64_t i = 0, j = 0; i < mb && j < mp;) {
      if (B[i].key < P[j].key) { i++; continue; }
      if (B[i].key > P[j].key) { j++; continue; }
      int64_t i2 = i, j2 = j;
      while (i2 < mb && B[i2].key == B[i].key) i2++;
      while (j2 < mp && P[j2].key == P[j].key) j2++;
      for (int64_t a = j; a < j2; a++)
        for (int64_t b = i; b < i2; b++) {
          out[w].probe = P[a].row;
          out[w].build = B[b].row;
          w++;
        }
      i = i2;
      j = j2;
    }
    qsort(out, (size_t)total, sizeof(pair_rows), cmp_pair);
    for (int64_t t = 0; t < keep; t++) {
      out_probe[t] = out[t].probe;
      out_build[t] = out[t].build;
    }
    free(out);
  }
  free(B);
  free(P);
  return total;
}

/* ---- hash partition ------------------------------------------------------ */

/* Partition id of every key: the top `bits` bits of k * 0x9E3779B97F4A7C15
 * (mod 2^64); 0 when bits == 0. */
void oc_partition_ids(const int64_t* keys, int64_t n, int32_t bits, int32_t* out_pid) {
  for (int64_t r = 0; r < n; r++) {
    uint64_t h = (uint64_t)keys[r] * 0x9E3779B97F4A7C15ULL;
    out_pid[r] = bits == 0 ? 0 : (int32_t)(h >> (64 - bits));
  }
}

/* Stable counting sort of the rows by partition id. out_perm[i] is the source
 * row of output position i; out_offsets has 2^bits + 1 entries. */
void oc_partition(const int64_t* keys, int64_t n, int32_t bits, int64_t* out_perm, int64_t* out_offsets) {
  int64_t parts = (int64_t)1 << bits;
  int32_t* pid = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  oc_partition_ids(keys, n, bits, pid);
  for (int64_t p = 0; p <= parts; p++) out_offsets[p] = 0;
  for (int64_t r = 0; r < n; r++) out_offsets[pid[r] + 1]++;
  for (int64_t p = 0; p < parts; p++) out_offsets[p + 1] += out_offsets[p];
  int64_t* cursor = (int64_t*)malloc((size_t)parts * sizeof(int64_t));
  memcpy(cursor, out_offsets, (size_t)parts * sizeof(int64_t));
  for (int64_t r = 0; r < n; r++) out_perm[cursor[pid[r]]++] = r;
  free(cursor);
  free(pid);
}

/* ---- NULLs ----------------------------------------------------------------
 * A column may carry a validity bitmap: bit r of byte r / 8, least significant
 * bit first, 1 when the value is present (the Arrow layout of the device
 * batches, Section 3.4); no bitmap means every value is present. SQL's
 * semantics, written out:
 *   selection   a predicate over a NULL value is not true, so the row does not
 *               pass (a conjunction passes only if every predicate is true)
 *   projection  a product with a NULL factor is NULL (a constant is never NULL)
 *   group-by    the rows whose key is NULL form one group of their own,
 *               emitted after every other group; COUNT(*) counts every row of
 *               a group; SUM_j and COUNT_j take only the rows whose e_j is not
 *               NULL; AVG_j = (double)SUM_j / (double)COUNT_j; SUM_j and AVG_j
 *               are NULL when COUNT_j is 0
 *   equi-join   a NULL key equals nothing, on either side
 */
static int valid_at(const uint8_t* v, int64_t r) { return v == NULL || ((v[r >> 3] >> (r & 7)) & 1); }

/* Selection with validity bitmaps (valid[c] NULL: column c has no NULLs). */
int64_t oc_filter_nullable(const oc_col* cols, const uint8_t* const* valid, int64_t n, int32_t np, const int32_t* pcol,
                           const int64_t* plo, const int64_t* phi, uint8_t* pass) {
  int64_t count = 0;
  for (int64_t r = 0; r < n; r++) {
    int ok = 1;
    for (int32_t j = 0; j < np && ok; j++) {
      if (!valid_at(valid[pcol[j]], r)) {
        ok = 0;
        break;
      }
      int64_t v = widen(&cols[pcol[j]], r);
      if (v < plo[j] || v > phi[j]) ok = 0;
    }
    pass[r] = (uint8_t)ok;
    count += ok;
  }
  return count;
}

/* Projection with validity: out_valid[r] (one byte per row) is 0 when a factor
 * reads a NULL value, and out[r] is then 0. */
void oc_project_nullable(const oc_col* cols, const uint8_t* const* valid, int64_t n, int32_t nf, const int32_t* fcol,
                         const int64_t* fsign, const int64_t* fadd, int64_t* out, uint8_t* out_valid) {
  for (int64_t r = 0; r < n; r++) {
    uint64_t acc = 1;
    int present = 1;
    for (int32_t f = 0; f < nf; f++) {
      int64_t x = 0;
      if (fcol[f] >= 0) {
        if (!valid_at(valid[fcol[f]], r)) present = 0;
        x = widen(&cols[fcol[f]], r);
      }
      uint64_t fac = (uint64_t)fsign[f] * (uint64_t)x + (uint64_t)fadd[f];
      acc = f == 0 ? fac : acc * fac;
    }
    out[r] = present ? (int64_t)acc : 0;
    out_valid[r] = (uint8_t)present;
  }
}

typedef struct {
  int64_t isnull, key, row;
} null_keyed_row;

static int cmp_null_keyed_row(const void* a, const void* b) {
  const null_keyed_row* x = (const null_keyed_row*)a;
  const null_keyed_row* y = (const null_keyed_row*)b;
  if (x->isnull != y->isnull) return x->isnull < y->isnull ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

/* Group-by over one key column that may hold NULLs (key_valid: a bitmap, or
 * NULL), with nval value arrays whose rows may be NULL (vals_valid[v]: one
 * byte per row, or NULL for none). Outputs per group g: out_keys[g] (0 for the
 * NULL group), out_key_null[g], out_count[g] = COUNT(*), and per value v at
 * g * nval + v: out_sums (0 when NULL), out_nonnull = COUNT_v, out_avg (0 when
 * NULL). Groups in ascending key order, the NULL group last. Returns the group
 * count, or -1 if it exceeds max_groups. */
int64_t oc_groupby_nullable(int64_t n, const uint8_t* pass, oc_col key, const uint8_t* key_valid, int32_t nval,
                            const int64_t* const* vals, const uint8_t* const* vals_valid, int64_t* out_keys,
                            uint8_t* out_key_null, int64_t* out_count, int64_t* out_sums, int64_t* out_nonnull,
                            double* out_avg, int64_t max_groups) {
  int64_t m = 0;
  for (int64_t r = 0; r < n; r++) m += (pass == NULL || pass[r]);
  null_keyed_row* rows = (null_keyed_row*)malloc((size_t)(m > 0 ? m : 1) * sizeof(null_keyed_row));
  int64_t w = 0;
  for (int64_t r = 0; r < n; r++) {
    if (pass != NULL && !pass[r]) continue;
    rows[w].isnull = !valid_at(key_valid, r);
    rows[w].key = rows[w].isnull ? 0 : widen(&key, r);
    rows[w].row = r;
    w++;
  }
  qsort(rows, (size_t)m, sizeof(null_keyed_row), cmp_null_keyed_row);
  int64_t g = 0;
  for (int64_t i = 0; i < m;) {
    int64_t j = i;
    while (j < m && rows[j].isnull == rows[i].isnull && rows[j].key == rows[i].key) j++;
    if (g >= max_groups) {
      free(rows);
      return -1;
    }
    out_keys[g] = rows[i].key;
    out_key_null[g] = (uint8_t)rows[i].isnull;
    out_count[g] = j - i;
    for (int32_t v = 0; v < nval; v++) {
      uint64_t s = 0;
      int64_t c = 0;
      for (int64_t t = i; t < j; t++) {
        const int64_t row = rows[t].row;
        if (vals_valid != NULL && vals_valid[v] != NULL && !vals_valid[v][row]) continue;
        s += (uint64_t)vals[v][row];
        c++;
      }
      out_sums[g * nval + v] = c ? (int64_t)s : 0;
      out_nonnull[g * nval + v] = c;
      out_avg[g * nval + v] = c ? (double)(int64_t)s / (double)c : 0.0;
    }
    g++;
    i = j;
  }
  free(rows);
  return g;
}

/* ---------------------------------------------------------------------------
 * Dictionary-encoded strings (Arrow dictionary arrays, Section 3.4). Two
 * string columns encoded against different dictionaries join on the strings
 * themselves: remap[i] is the index of the build dictionary entry whose bytes
 * equal probe dictionary entry i, or -1 when there is none. Definition
 * written out: the build entries are sorted by (length, bytes) and each
 * probe entry is looked up by binary search with the same order.
 */
typedef struct {
  const int32_t* off;
  const uint8_t* data;
} str_col;

static int cmp_str(const str_col* c, int64_t i, const uint8_t* s, int32_t len) {
  const int32_t a = c->off[i], li = c->off[i + 1] - a;
  if (li != len) return li < len ? -1 : 1;
  return len ? memcmp(c->data + a, s, (size_t)len) : 0;
}

static const str_col* g_sort_col;
static int cmp_str_idx(const void* x, const void* y) {
  const int64_t j = *(const int64_t*)y;
  const int32_t a = g_sort_col->off[j];
  return cmp_str(g_sort_col, *(const int64_t*)x, g_sort_col->data + a, g_sort_col->off[j + 1] - a);
}

void oc_dict_unify(const int32_t* boff, const uint8_t* bdata, int64_t nb, const int32_t* poff, const uint8_t* pdata,
                   int64_t np, int32_t* remap) {
  str_col b = {boff, bdata};
  int64_t* idx = (int64_t*)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < nb; i++) idx[i] = i;
  g_sort_col = &b;
  qsort(idx, (size_t)nb, sizeof(int64_t), cmp_str_idx);
  for (int64_t i = 0; i < np; i++) {
    const uint8_t* s = pdata + poff[i];
    const int32_t len = poff[i + 1] - poff[i];
    int64_t lo = 0, hi = nb;
    remap[i] = -1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      const int c = cmp_str(&b, idx[mid], s, len);
      if (c == 0) {
        remap[i] = (int32_t)idx[mid];
        break;
      }
      if (c < 0) lo = mid + 1;
      else hi = mid;
    }
  }
  free(idx);
}
