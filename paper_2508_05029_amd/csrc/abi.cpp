// Status codes, thread-local error text and argument validation of the C ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "common.h"

namespace tq {

static thread_local char g_last_error[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
}

tq_status fail(tq_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return s;
}

tq_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return TQ_EHIP;
}

int device_cu_count() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

static bool valid_type(int32_t t) { return t == TQ_U8 || t == TQ_I32 || t == TQ_I64; }

tq_status make_plan(RowPlan* P, const tq_col* in, int32_t ncol, const tq_pred* p, int32_t np, const tq_expr* e,
                    int32_t ne, const tq_gkey* key, int64_t nrows, bool allow_nulls) {
  *P = RowPlan{};
  if (nrows < 0) return fail(TQ_EINVAL, "nrows < 0");
  if (ncol < 0 || ncol > TQ_MAX_COLS) return fail(TQ_EINVAL, "ncol %d outside [0, %d]", ncol, TQ_MAX_COLS);
  if (np < 0 || np > TQ_MAX_PREDS) return fail(TQ_EINVAL, "np %d outside [0, %d]", np, TQ_MAX_PREDS);
  if (ne < 0 || ne > TQ_MAX_SUMS) return fail(TQ_EINVAL, "expression count %d outside [0, %d]", ne, TQ_MAX_SUMS);
  if (ncol > 0 && in == nullptr) return fail(TQ_EINVAL, "columns are NULL");
  if (np > 0 && p == nullptr) return fail(TQ_EINVAL, "predicates are NULL");
  if (ne > 0 && e == nullptr) return fail(TQ_EINVAL, "expressions are NULL");
  P->ncol = ncol;
  for (int c = 0; c < ncol; c++) {
    if (!valid_type(in[c].type)) return fail(TQ_EINVAL, "column %d: bad type %d", c, in[c].type);
    if (nrows > 0 && in[c].data == nullptr) return fail(TQ_EINVAL, "column %d: NULL data", c);
    if (((uintptr_t)in[c].data & 15) != 0) return fail(TQ_EINVAL, "column %d: not 16-byte aligned", c);
    if (in[c].valid && !allow_nulls)
      return fail(TQ_EINVAL, "column %d has a validity bitmap: use the _nullable entry point", c);
    P->col[c].p = in[c].data;
    P->col[c].w = in[c].type;
    P->col[c].valid = in[c].valid;
  }
  P->np = np;
  for (int j = 0; j < np; j++) {
    if (p[j].col < 0 || p[j].col >= ncol) return fail(TQ_EINVAL, "predicate %d: column %d out of range", j, p[j].col);
    P->pred[j].mask = 1u << p[j].col;
    P->pred[j].lo = p[j].lo;
    P->pred[j].hi = p[j].hi;
  }
  P->ne = ne;
  for (int j = 0; j < ne; j++) {
    if (e[j].nf < 1 || e[j].nf > 3) return fail(TQ_EINVAL, "expression %d: %d factors (1..3)", j, e[j].nf);
    P->expr[j].nf = e[j].nf;
    for (int f = 0; f < e[j].nf; f++) {
      const tq_factor& F = e[j].f[f];
      if (F.col < -1 || F.col >= ncol) return fail(TQ_EINVAL, "expression %d factor %d: column %d", j, f, F.col);
      P->expr[j].f[f] = make_factor(F.col, F.sign, F.add);
    }
  }
  if (key) {
    if (key->ncol < 1 || key->ncol > 2) return fail(TQ_EINVAL, "group key: %d columns (1..2)", key->ncol);
    for (int c = 0; c < key->ncol; c++)
      if (key->col[c] < 0 || key->col[c] >= ncol) return fail(TQ_EINVAL, "group key column %d", key->col[c]);
    P->key_ncol = key->ncol;
    P->key_mask[0] = 1u << key->col[0];
    P->key_mask[1] = key->ncol == 2 ? 1u << key->col[1] : 0u;
    P->key_mult = key->mult;
  }
  // keep only the columns a predicate, expression or key reads, so that the
  // kernels load nothing else; masks are renumbered to the kept columns
  uint32_t used = P->key_mask[0] | P->key_mask[1];
  for (int j = 0; j < P->np; j++) used |= P->pred[j].mask;
  for (int j = 0; j < P->ne; j++)
    for (int f = 0; f < P->expr[j].nf; f++) used |= P->expr[j].f[f].mask;
  uint32_t remap[TQ_MAX_COLS];
  int kept = 0;
  for (int c = 0; c < ncol; c++) {
    remap[c] = 0;
    if ((used >> c) & 1u) {
      P->col[kept] = P->col[c];
      remap[c] = 1u << kept;
      kept++;
    }
  }
  for (int c = kept; c < ncol; c++) P->col[c] = DCol{nullptr, 0, nullptr};
  P->null_cols = 0;
  for (int c = 0; c < kept; c++) P->null_cols |= (P->col[c].valid ? 1u : 0u) << c;
  auto re = [&](uint32_t m) -> uint32_t { return m ? remap[__builtin_ctz(m)] : 0u; };
  for (int j = 0; j < P->np; j++) P->pred[j].mask = re(P->pred[j].mask);
  for (int j = 0; j < P->ne; j++)
    for (int f = 0; f < P->expr[j].nf; f++) P->expr[j].f[f].mask = re(P->expr[j].f[f].mask);
  P->key_mask[0] = re(P->key_mask[0]);
  P->key_mask[1] = re(P->key_mask[1]);
  P->ncol = kept;
  return TQ_OK;
}

}  // namespace tq

extern "C" {

const char* tq_strerror(tq_status s) {
  switch (s) {
    case TQ_OK: return "ok";
    case TQ_EINVAL: return "invalid argument";
    case TQ_ENOMEM: return "out of pool pages or device budget";
    case TQ_EFULL: return "hash table or output capacity too small";
    case TQ_EDOMAIN: return "group key outside its domain";
    case TQ_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* tq_last_error(void) { return tq::g_last_error; }

int32_t tq_version(void) { return 1; }

}  // extern "C"
