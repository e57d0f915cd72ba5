// Shared device and host definitions of libtq (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tq.h"

namespace tq {

constexpr uint64_t kFib = 0x9E3779B97F4A7C15ull;  // floor(2^64 / golden ratio)
constexpr int kWave = 64;
constexpr int kRows = 4;  // rows per thread per step of the streaming kernels

// ---------------------------------------------------------------- host side

void set_error(const char* fmt, ...);
tq_status fail(tq_status s, const char* fmt, ...);
tq_status hip_fail(hipError_t e, const char* what);
int device_cu_count();

#define TQ_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::tq::hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------- plan descriptors
// Passed to kernels by value. Columns widen to int64.

struct DCol {
  const void* p;
  int32_t w;  // byte width 1, 4 or 8
};

struct DPred {
  int32_t col;
  int64_t lo, hi;
};

struct DFactor {
  int32_t col;  // -1: constant
  int64_t sign;
  int64_t add;
};

struct DExpr {
  int32_t nf;
  DFactor f[3];
};

struct RowPlan {
  DCol col[TQ_MAX_COLS];
  int32_t ncol;
  DPred pred[TQ_MAX_PREDS];
  int32_t np;
  DExpr expr[TQ_MAX_SUMS];
  int32_t ne;
  int32_t key_ncol;  // group key (0 when unused)
  int32_t key_col[2];
  int64_t key_mult;
};

// Validates and copies host descriptors into a RowPlan. Returns TQ_OK or TQ_EINVAL.
tq_status make_plan(RowPlan* plan, const tq_col* in, int32_t ncol, const tq_pred* p, int32_t np,
                    const tq_expr* e, int32_t ne, const tq_gkey* key, int64_t nrows);

// ------------------------------------------------------- object headers

constexpr uint32_t kTableMagic = 0x54514A54u;  // "TJQT"
constexpr uint32_t kStateMagic = 0x54514753u;  // "SGQT"
constexpr size_t kHeaderBytes = 256;

struct TableHeader {
  uint32_t magic;
  int32_t err;
  int64_t cap_max;   // slots available in the buffer (power of two)
  int32_t log2cap;   // slots used by the current build
  int32_t skip;      // high hash bits ignored by the slot index
  int64_t n;         // rows inserted by the current build
  int64_t n_acc;     // counting accumulator (self-resetting)
  uint32_t ticket;   // last-block ticket (self-resetting)
  uint32_t flags;
  double lf;
};
static_assert(sizeof(TableHeader) <= kHeaderBytes, "header");

struct StateHeader {
  uint32_t magic;
  int32_t err;
  int64_t domain;
  int32_t nsum;
  int32_t replicas;  // power of two; replica r of entry e at data[r * domain * stride + e]
  int64_t matches;   // unused by the kernels; reserved
};
static_assert(sizeof(StateHeader) <= kHeaderBytes, "header");

__host__ __device__ inline uint32_t* table_tags(void* t) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t) + kHeaderBytes);
}
__host__ __device__ inline int64_t* table_slots(void* t, int64_t cap_max) {
  size_t tag_bytes = ((size_t)cap_max * 4 + 255) & ~(size_t)255;
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(t) + kHeaderBytes + tag_bytes);
}
__host__ __device__ inline int64_t* state_data(void* s) {
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(s) + kHeaderBytes);
}

// ------------------------------------------------------- device helpers

__device__ __forceinline__ void latch_error(int32_t* err, int32_t code) { atomicCAS(err, 0, code); }

__device__ __forceinline__ uint64_t mulhash(int64_t k) { return (uint64_t)k * kFib; }

// Tag of a hash: its low 32 bits, with 0 reserved for "empty".
__device__ __forceinline__ uint32_t hash_tag(uint64_t h) {
  uint32_t t = (uint32_t)h;
  return t ? t : 1u;
}

__device__ __forceinline__ uint64_t slot_of(uint64_t h, int skip, int log2cap) {
  return (h << skip) >> (64 - log2cap);
}

template <typename T>
__device__ __forceinline__ T ntload(const T* p) {
  return __builtin_nontemporal_load(p);
}

// Widened load of one value.
__device__ __forceinline__ int64_t load1(const DCol& c, int64_t r) {
  if (c.w == 8) return ntload(static_cast<const int64_t*>(c.p) + r);
  if (c.w == 4) return (int64_t)ntload(static_cast<const int32_t*>(c.p) + r);
  return (int64_t)ntload(static_cast<const uint8_t*>(c.p) + r);
}

typedef long long v2i64 __attribute__((ext_vector_type(2)));
typedef int v4i32 __attribute__((ext_vector_type(4)));

// kRows consecutive values starting at row r0 (a multiple of kRows); `full`
// means all kRows rows exist. Column pointers are 16-byte aligned.
__device__ __forceinline__ void load4(const DCol& c, int64_t r0, bool full, int64_t n, int64_t (&v)[kRows]) {
  if (full) {
    if (c.w == 8) {
      const v2i64* q = reinterpret_cast<const v2i64*>(static_cast<const int64_t*>(c.p) + r0);
      v2i64 a = ntload(q), b = ntload(q + 1);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if (c.w == 4) {
      v4i32 a = ntload(reinterpret_cast<const v4i32*>(static_cast<const int32_t*>(c.p) + r0));
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
      uint32_t a = ntload(reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(c.p) + r0));
      v[0] = a & 0xff; v[1] = (a >> 8) & 0xff; v[2] = (a >> 16) & 0xff; v[3] = a >> 24;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kRows; i++) v[i] = (r0 + i < n) ? load1(c, r0 + i) : 0;
  }
}

// Value of column `idx` among the loaded ones (idx is uniform).
__device__ __forceinline__ int64_t pick(const int64_t (&vals)[TQ_MAX_COLS], int idx) {
  int64_t r = vals[0];
#pragma unroll
  for (int i = 1; i < TQ_MAX_COLS; i++) r = (idx == i) ? vals[i] : r;
  return r;
}

__device__ __forceinline__ bool eval_preds(const RowPlan& P, const int64_t (&vals)[TQ_MAX_COLS]) {
  bool ok = true;
  for (int j = 0; j < P.np; j++) {
    int64_t x = pick(vals, P.pred[j].col);
    ok = ok && (x >= P.pred[j].lo) && (x <= P.pred[j].hi);
  }
  return ok;
}

__device__ __forceinline__ int64_t eval_expr(const DExpr& E, const int64_t (&vals)[TQ_MAX_COLS]) {
  uint64_t acc = 1;
  for (int f = 0; f < E.nf; f++) {
    int64_t x = E.f[f].col < 0 ? 0 : pick(vals, E.f[f].col);
    uint64_t fac = (uint64_t)E.f[f].sign * (uint64_t)x + (uint64_t)E.f[f].add;
    acc = f == 0 ? fac : acc * fac;
  }
  return (int64_t)acc;
}

__device__ __forceinline__ int64_t eval_key(const RowPlan& P, const int64_t (&vals)[TQ_MAX_COLS]) {
  int64_t k = pick(vals, P.key_col[0]);
  if (P.key_ncol == 2) k = (int64_t)((uint64_t)k * (uint64_t)P.key_mult + (uint64_t)pick(vals, P.key_col[1]));
  return k;
}

// Inclusive prefix sum over the wave of a 32-bit value; returns the exclusive
// prefix and sets *total to the wave sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t* total) {
  int lane = __lane_id();
  uint32_t s = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(s, d, kWave);
    if (lane >= d) s += y;
  }
  *total = __shfl(s, kWave - 1, kWave);
  return s - x;
}

}  // namespace tq
