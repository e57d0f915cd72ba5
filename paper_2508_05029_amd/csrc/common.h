// Shared device and host definitions of libtq (gfx950, wave64).
//
// Design rules that the kernels follow on MI355X:
//   * no contended device-scope atomics and no __threadfence on hot paths:
//     a device-scope atomic on one address serialises across the 8 XCDs and a
//     release fence writes back the XCD's L2; per-workgroup partials plus a
//     scan or a fold in the next kernel take their place
//   * LDS atomics go through __shared__-typed pointers (ds_* instructions,
//     never flat atomics)
//   * the kernels are instantiated for the number of columns a query reads
//     (NC), so that the loaded rows stay in registers
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

// A run of `npages` consecutive free pages of the pool (one contiguous host
// range, pinned when the pool is): *first gets the first page's id. The
// library's own host staging (descriptor uploads, counts read back) comes from
// here, so that no call pins memory of its own. TQ_ENOMEM if no run is free.
tq_status pool_take_run(tq_pagepool* pool, int64_t npages, int32_t* first);
void pool_give_run(tq_pagepool* pool, int32_t first, int64_t npages);

#define TQ_HIP(call)                                        \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::tq::hip_fail(e_, #call); \
  } while (0)

// Smallest supported column-count bucket >= ncol.
inline int nc_bucket(int ncol) { return ncol <= 1 ? 1 : ncol <= 2 ? 2 : ncol <= 4 ? 4 : 8; }

#define TQ_DISPATCH_NC(ncol, NCV, ...)                  \
  switch (::tq::nc_bucket(ncol)) {                      \
    case 1: { constexpr int NCV = 1; __VA_ARGS__; break; } \
    case 2: { constexpr int NCV = 2; __VA_ARGS__; break; } \
    case 4: { constexpr int NCV = 4; __VA_ARGS__; break; } \
    default: { constexpr int NCV = 8; __VA_ARGS__; break; } \
  }

// ------------------------------------------------------- plan descriptors
// Passed to kernels by value. Columns widen to int64.

struct DCol {
  const void* p;
  int32_t w;  // byte width 1, 4 or 8
  const uint8_t* valid = nullptr;  // validity bitmap (bit r of byte r / 8), or none
};

// Columns are referenced through one-bit masks (bit c = plan column c; 0 = the
// constant 0), which the kernels resolve with a short chain of selects.
struct DPred {
  uint32_t mask;
  int64_t lo, hi;
};

struct DFactor {
  uint32_t mask;  // 0: the factor is the constant `add` (and `sign` is 0)
  int64_t sign;
  int64_t add;
};

// A factor over column `col` (or the constant `add` when col < 0, whose sign
// is zeroed so that whatever column value a kernel picks for it drops out).
inline DFactor make_factor(int col, int64_t sign, int64_t add) {
  return DFactor{col < 0 ? 0u : 1u << col, col < 0 ? 0 : sign, add};
}

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
  uint32_t key_mask[2];
  int64_t key_mult;
  uint32_t null_cols;  // bit c: plan column c carries a validity bitmap
};

// Validates and copies host descriptors into a RowPlan. Returns TQ_OK or
// TQ_EINVAL (also for a column with a validity bitmap unless allow_nulls).
tq_status make_plan(RowPlan* plan, const tq_col* in, int32_t ncol, const tq_pred* p, int32_t np,
                    const tq_expr* e, int32_t ne, const tq_gkey* key, int64_t nrows, bool allow_nulls = false);

// ------------------------------------------------------- object headers

constexpr uint32_t kTableMagic = 0x54514A54u;
constexpr uint32_t kStateMagic = 0x54514753u;
constexpr uint32_t kScanMagic = 0x54515053u;  // a Parquet decode's work buffer
constexpr size_t kHeaderBytes = 256;
constexpr int kMaxPartBlocks = 2048;  // per-block partial counts kept in a table

struct TableHeader {
  uint32_t magic;
  int32_t err;
  int64_t cap_max;   // slots available in the buffer (power of two)
  int32_t log2cap;   // slots used by the current build
  int32_t skip;      // high hash bits ignored by the slot index
  int64_t n;         // rows inserted by the current build
  int32_t nblk;      // blocks that wrote partial counts
  uint32_t flags;
  double lf;
  int32_t log2g;     // buckets per region (log2): linear probing wraps inside a region
  int32_t regions;   // 1: the last build filled each region in LDS; 0: it inserted with global CAS
  int32_t alt;       // 1: the tags and slots in use are the build scratch's (see scratch_alt_tags)
  int32_t ovf;       // set during a build when a region's rows do not fit it
  int32_t bloom_log2w;  // the build's Bloom filter has 2^bloom_log2w 32-bit words; 0: none
};
static_assert(sizeof(TableHeader) <= kHeaderBytes, "header");

struct StateHeader {
  uint32_t magic;
  int32_t err;
  int64_t domain;
  int32_t nsum;
  int32_t rows;  // partial rows: > 1 for block-private partials, 1 for one shared table
  int64_t used;  // private rows written since init (the largest grid of an aggregating launch)
  int32_t nullable;  // 1: groups [0, domain - 1) and the NULL group domain - 1; per sum SUM_j, COUNT_j
};
static_assert(sizeof(StateHeader) <= kHeaderBytes, "header");

// Table: header | int64 partial[kMaxPartBlocks] | uint16 tag[cap_max] |
// {key, payload}[cap_max] | build scratch (the region build's tickets, bin
// counts and row segments; see table_scratch).
// Slots form buckets of kBucket; the 16-bit tags of one bucket are one 16-byte
// word group, read with a single load.
constexpr int kBucket = 8;
constexpr int kLog2Bucket = 3;

__host__ __device__ inline size_t table_tag_bytes(int64_t cap_max) {
  return ((size_t)cap_max * 2 + 255) & ~(size_t)255;
}
__host__ __device__ inline int64_t* table_partials(void* t) {
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(t) + kHeaderBytes);
}
// Tag words: two 16-bit tags per uint32, bucket b = words [4b, 4b + 4).
__host__ __device__ inline uint32_t* table_tags(void* t) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(t) + kHeaderBytes + kMaxPartBlocks * 8);
}
__host__ __device__ inline int64_t* table_slots(void* t, int64_t cap_max) {
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(t) + kHeaderBytes + kMaxPartBlocks * 8 +
                                    table_tag_bytes(cap_max));
}
// Region build scratch, after the slots, sized by the capacity: int32
// block_rows[max_grid] | uint32 meta[max_grid][kMetaStride] ((offset << 16) |
// count of one block's rows in each region; rows padded past kRegionBins so
// that one region's counts over the blocks do not all fall in the same cache
// channels) | {key, payload}[cap_max] (each
// block's passing rows, grouped by region, at block * kPartRows) | uint16
// alt_tags[cap_max], where max_grid = part_grid_max(cap_max). When a region
// overflows, the fallback insert builds the whole table into alt_tags and
// the row area (which then serves as the slots). Then uint64
// bloom[bloom_words_max(cap_max)]: a region build's Bloom filter, one block of
// 2^bloom_log2w / kRegionBins words per region.
constexpr int kRegionBins = 256;  // the top 8 bits of a bucket index select its region
constexpr int kLog2Bins = 8;
constexpr int kPartBlock = 512;
constexpr int kPartSub = 1;                              // groups of kRows rows per thread
constexpr int kPartRows = kPartBlock * kRows * kPartSub;  // rows per partitioning block
constexpr int kMetaStride = kRegionBins + 8;
__host__ __device__ inline int64_t part_grid_max(int64_t cap_max) {
  return cap_max / kPartRows > 1 ? cap_max / kPartRows : 1;
}
__host__ __device__ inline size_t block_rows_bytes(int64_t cap_max) {
  return ((size_t)part_grid_max(cap_max) * 4 + 255) & ~(size_t)255;
}
// Bloom words (32-bit) for a table of `cap` slots: two bits per slot, between
// two words per region and 2 MiB. Up to 128 KiB (the LDS a probe workgroup
// gives it) a probe reads the filter from LDS, past that from device memory,
// where one XCD's 4 MiB L2 can hold it.
constexpr int kBloomWordsMax = 32768;
constexpr int kLog2BloomWordsMax = 15;
constexpr int kGBloomWordsMax = 1 << 19;
constexpr int kLog2GBloomWordsMax = 19;
__host__ __device__ inline int64_t bloom_words_max(int64_t cap) {
  const int64_t w = cap / 16;
  return w < 2 * kRegionBins ? 2 * kRegionBins : (w > kGBloomWordsMax ? kGBloomWordsMax : w);
}
__host__ __device__ inline size_t scratch_bytes(int64_t cap_max) {
  return block_rows_bytes(cap_max) + (size_t)part_grid_max(cap_max) * kMetaStride * 4 + (size_t)cap_max * 16 +
         table_tag_bytes(cap_max) + (size_t)bloom_words_max(cap_max) * 4;
}
__host__ __device__ inline char* table_scratch(void* t, int64_t cap_max) {
  return reinterpret_cast<char*>(table_slots(t, cap_max)) + (size_t)cap_max * 16;
}
__host__ __device__ inline int32_t* scratch_block_rows(void* t, int64_t cap_max) {
  return reinterpret_cast<int32_t*>(table_scratch(t, cap_max));
}
__host__ __device__ inline uint32_t* scratch_meta(void* t, int64_t cap_max) {
  return reinterpret_cast<uint32_t*>(table_scratch(t, cap_max) + block_rows_bytes(cap_max));
}
__host__ __device__ inline int64_t* scratch_rows(void* t, int64_t cap_max) {
  return reinterpret_cast<int64_t*>(scratch_meta(t, cap_max) + (size_t)part_grid_max(cap_max) * kMetaStride);
}
__host__ __device__ inline uint32_t* scratch_alt_tags(void* t, int64_t cap_max) {
  return reinterpret_cast<uint32_t*>(scratch_rows(t, cap_max) + (size_t)cap_max * 2);
}
__host__ __device__ inline uint32_t* scratch_bloom(void* t, int64_t cap_max) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(scratch_alt_tags(t, cap_max)) + table_tag_bytes(cap_max));
}
__host__ __device__ inline int64_t* state_data(void* s) {
  return reinterpret_cast<int64_t*>(reinterpret_cast<char*>(s) + kHeaderBytes);
}

// ------------------------------------------------------- device helpers

__device__ __forceinline__ void latch_error(int32_t* err, int32_t code) { atomicCAS(err, 0, code); }

__device__ __forceinline__ uint64_t mulhash(int64_t k) { return (uint64_t)k * kFib; }

// Tag of a hash: its low 16 bits, with 0 reserved for "empty".
__device__ __forceinline__ uint32_t hash_tag(uint64_t h) {
  uint32_t t = (uint32_t)h & 0xffffu;
  return t ? t : 1u;
}

// Home bucket: the high bits of the hash below the `skip` partition bits.
__device__ __forceinline__ uint64_t bucket_of(uint64_t h, int skip, int log2buckets) {
  return (h << skip) >> (64 - log2buckets);
}

// Whether hash h belongs to the partition a table was built for
// (TQ_SELECT_PARTITION: partition id = flags >> 16 in the top `skip` bits).
__device__ __forceinline__ bool in_partition(uint64_t h, int skip, uint32_t flags) {
  return !(flags & TQ_SELECT_PARTITION) || (uint32_t)(h >> (64 - skip)) == (flags >> 16);
}

// Bloom filter of a region-built table, from the key's multiplicative hash h:
// the key's region (as for its bucket) selects a block of 2^(log2w -
// kLog2Bins) 32-bit words, bits 19.. of h the word in the block and three bit
// positions in it, from the bits above those (from bit 26 at least): bits
// that the tag, the slot start and the bucket index of tables up to 2^(23 -
// skip) buckets leave unused (the largest filters share one or two with the
// bucket index of the largest tables).
__device__ __forceinline__ uint32_t bloom_word(uint64_t h, int skip, int log2w) {
  const uint32_t region = (uint32_t)((h << skip) >> (64 - kLog2Bins));
  const int sub_bits = log2w - kLog2Bins;
  const uint32_t sub = (uint32_t)(h >> 19) & ((1u << sub_bits) - 1u);
  return (region << sub_bits) | sub;
}
__device__ __forceinline__ uint32_t bloom_bits(uint64_t h, int log2w = kLog2BloomWordsMax) {
  const int sub_bits = log2w - kLog2Bins;
  const uint32_t x = (uint32_t)(h >> (sub_bits > 7 ? 19 + sub_bits : 26));
  return (1u << (x & 31u)) | (1u << ((x >> 5) & 31u)) | (1u << ((x >> 10) & 31u));
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

// R (2 or 4) consecutive values starting at row r0 (a multiple of R); `full`
// means all R rows exist. Column pointers are 16-byte aligned.
template <int R = kRows>
__device__ __forceinline__ void load4(const DCol& c, int64_t r0, bool full, int64_t n, int64_t (&v)[R]) {
  static_assert(R == 2 || R == 4, "rows per thread");
  if (full) {
    if (c.w == 8) {
      const v2i64* q = reinterpret_cast<const v2i64*>(static_cast<const int64_t*>(c.p) + r0);
#pragma unroll
      for (int h = 0; h < R / 2; h++) {
        v2i64 a = ntload(q + h);
        v[2 * h] = a.x;
        v[2 * h + 1] = a.y;
      }
    } else if (c.w == 4) {
      if (R == 4) {
        v4i32 a = ntload(reinterpret_cast<const v4i32*>(static_cast<const int32_t*>(c.p) + r0));
        v[0] = a.x; v[1] = a.y; v[R > 2 ? 2 : 0] = a.z; v[R > 2 ? 3 : 1] = a.w;
      } else {
        uint64_t a = ntload(reinterpret_cast<const uint64_t*>(static_cast<const int32_t*>(c.p) + r0));
        v[0] = (int32_t)(uint32_t)a;
        v[1] = (int32_t)(uint32_t)(a >> 32);
      }
    } else {
      if (R == 4) {
        uint32_t a = ntload(reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(c.p) + r0));
#pragma unroll
        for (int i = 0; i < R; i++) v[i] = (a >> (8 * i)) & 0xff;
      } else {
        uint32_t a = ntload(reinterpret_cast<const uint16_t*>(static_cast<const uint8_t*>(c.p) + r0));
        v[0] = a & 0xff;
        v[1] = (a >> 8) & 0xff;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; i++) v[i] = (r0 + i < n) ? load1(c, r0 + i) : 0;
  }
}

// Raw bytes of R (2 or 4) consecutive values of one column, loaded but not
// yet widened, with the same instructions for every width: the 16-byte block
// that holds row r0 (for R = 4 and 8-byte values, also the next one; for
// other widths that load repeats the first). A column's width is only known
// at run time, and a load in a branch of the width puts a wait inside the
// branch, one memory latency per column; so every column is loaded before
// any is widened. The caller makes sure rows r0 .. r0 + 15 exist, so that
// the blocks lie inside the column (columns are 16-byte aligned).
struct RawCol {
  v4i32 a, b;
  uint32_t off;  // byte offset of row r0 in block a
};

template <int R>
__device__ __forceinline__ void load_raw(const DCol& c, int64_t r0, RawCol& x) {
  // pointer arithmetic on the column pointer (an integer round trip would
  // lose its address space and turn the loads into flat loads)
  const char* at = static_cast<const char*>(c.p) + r0 * c.w;
  x.off = (uint32_t)(reinterpret_cast<uintptr_t>(at) & 15);
  const v4i32* blk = reinterpret_cast<const v4i32*>(at - x.off);
  x.a = ntload(blk);
  if (R == 4) x.b = ntload(blk + (c.w == 8 ? 1 : 0));
}

__device__ __forceinline__ uint32_t word_at(const v4i32& a, uint32_t q) {
  uint32_t r = (uint32_t)a.x;
  r = q == 1 ? (uint32_t)a.y : r;
  r = q == 2 ? (uint32_t)a.z : r;
  r = q == 3 ? (uint32_t)a.w : r;
  return r;
}

template <int R>
__device__ __forceinline__ void widen_raw(const DCol& c, const RawCol& x, int64_t (&v)[R]) {
  if (c.w == 8) {  // block-aligned: R = 2 fills a, R = 4 fills a and b
    v[0] = (int64_t)(((uint64_t)(uint32_t)x.a.y << 32) | (uint32_t)x.a.x);
    v[1] = (int64_t)(((uint64_t)(uint32_t)x.a.w << 32) | (uint32_t)x.a.z);
    if (R == 4) {
      v[R > 2 ? 2 : 0] = (int64_t)(((uint64_t)(uint32_t)x.b.y << 32) | (uint32_t)x.b.x);
      v[R > 2 ? 3 : 1] = (int64_t)(((uint64_t)(uint32_t)x.b.w << 32) | (uint32_t)x.b.z);
    }
  } else if (c.w == 4) {  // R = 4: block-aligned; R = 2: at word 0 or 2
    const uint32_t q = x.off >> 2;
#pragma unroll
    for (int i = 0; i < R; i++) v[i] = (int32_t)word_at(x.a, q + i);
  } else {  // 1 byte: R bytes inside one word of the block
    const uint32_t wv = word_at(x.a, x.off >> 2) >> (8 * (x.off & 3));
#pragma unroll
    for (int i = 0; i < R; i++) v[i] = (wv >> (8 * i)) & 0xff;
  }
}

// The rows r0..r0+R-1 of the first NC plan columns: v[c][i].
template <int NC, int R = kRows>
__device__ __forceinline__ void load_rows(const RowPlan& P, int64_t r0, bool full, int64_t n, int64_t (&v)[NC][R]) {
  if (r0 + 16 <= n) {
    RawCol raw[NC];
#pragma unroll
    for (int c = 0; c < NC; c++)
      if (c < P.ncol) load_raw<R>(P.col[c], r0, raw[c]);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if (c < P.ncol) widen_raw<R>(P.col[c], raw[c], v[c]);
      else {
#pragma unroll
        for (int i = 0; i < R; i++) v[c][i] = 0;
      }
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < NC; c++) {
    if (c < P.ncol) load4<R>(P.col[c], r0, false, n, v[c]);
    else {
#pragma unroll
      for (int i = 0; i < R; i++) v[c][i] = 0;
    }
  }
}

// As load_rows for plan columns that are all 8 bytes wide and rows that all
// exist: one 16-byte load per column and row pair, with no branch between the
// loads (a branch on the width puts a wait for each load inside it).
template <int NC, int R = kRows>
__device__ __forceinline__ void load_rows64(const RowPlan& P, int64_t r0, int64_t (&v)[NC][R]) {
#pragma unroll
  for (int c = 0; c < NC; c++) {
    if (c < P.ncol) {
      const v2i64* q = reinterpret_cast<const v2i64*>(static_cast<const int64_t*>(P.col[c].p) + r0);
#pragma unroll
      for (int h = 0; h < R / 2; h++) {
        const v2i64 a = ntload(q + h);
        v[c][2 * h] = a.x;
        v[c][2 * h + 1] = a.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; i++) v[c][i] = 0;
    }
  }
}

// Value of the column selected by `mask` (one bit, uniform) for row i; 0 if mask is 0.
template <int NC, int R>
__device__ __forceinline__ int64_t pick(const int64_t (&v)[NC][R], int i, uint32_t mask) {
  // The column index is the same in every lane, so a wider row is indexed
  // directly (the compiler moves the row's registers by the index held in a
  // scalar register) instead of through one select per column, whose lane
  // masks, kept live across a kernel's loop, spill. A zero mask (a constant
  // factor, whose sign is zero) reads the last column.
  // (Up to two columns the plain chain is kept: in the pipelined probe the
  // other forms raised register pressure into scratch spills.)
  static_assert(NC <= 8, "pick: at most 8 columns");
  if constexpr (NC <= 2) {
    int64_t r = 0;
#pragma unroll
    for (int c = 0; c < NC; c++) r = ((mask >> c) & 1u) ? v[c][i] : r;
    return r;
  } else {
    const uint32_t c = min((uint32_t)__builtin_ctz(mask | 0x80000000u), (uint32_t)NC - 1);
    int64_t t[NC];
#pragma unroll
    for (int k = 0; k < NC; k++) t[k] = v[k][i];
    return t[c];
  }
}

// A rolled loop over the plan's predicates: unrolled over TQ_MAX_PREDS, the
// bounds of all of them stay live in scalar registers across a kernel's main
// loop and spill into vector lanes that every row then reads back.
template <int NC, int R>
__device__ __forceinline__ bool eval_preds(const RowPlan& P, const int64_t (&v)[NC][R], int i) {
  bool ok = true;
#pragma unroll 1
  for (int j = 0; j < P.np; j++) {
    int64_t x = pick<NC, R>(v, i, P.pred[j].mask);
    ok = ok && (x >= P.pred[j].lo) && (x <= P.pred[j].hi);
  }
  return ok;
}

template <int NC, int R>
__device__ __forceinline__ int64_t eval_expr(const DExpr& E, const int64_t (&v)[NC][R], int i) {
  uint64_t acc = 1;
#pragma unroll
  for (int f = 0; f < 3; f++) {
    if (f < E.nf) {
      int64_t x = pick<NC, R>(v, i, E.f[f].mask);
      uint64_t fac = (uint64_t)E.f[f].sign * (uint64_t)x + (uint64_t)E.f[f].add;
      acc = f == 0 ? fac : acc * fac;
    }
  }
  return (int64_t)acc;
}

template <int NC, int R>
__device__ __forceinline__ int64_t eval_key(const RowPlan& P, const int64_t (&v)[NC][R], int i) {
  int64_t k = pick<NC, R>(v, i, P.key_mask[0]);
  if (P.key_ncol == 2) k = (int64_t)((uint64_t)k * (uint64_t)P.key_mult + (uint64_t)pick<NC, R>(v, i, P.key_mask[1]));
  return k;
}

// ----------------------------------------------------------------- NULLs

__device__ __forceinline__ bool bit_at(const uint8_t* v, int64_t r) { return (v[r >> 3] >> (r & 7)) & 1u; }

// The plan columns present at row r, as a mask (bit c set: column c is not
// NULL there).
template <int NC>
__device__ __forceinline__ uint32_t row_present(const RowPlan& P, int64_t r) {
  uint32_t m = ~0u;
#pragma unroll
  for (int c = 0; c < NC; c++)
    if ((P.null_cols >> c) & 1u) m &= ~((uint32_t)!bit_at(P.col[c].valid, r) << c);
  return m;
}

// Every predicate true, none over a NULL value (a predicate over NULL is not true).
template <int NC, int R>
__device__ __forceinline__ bool eval_preds_present(const RowPlan& P, const int64_t (&v)[NC][R], int i,
                                                   uint32_t present) {
  bool ok = true;
#pragma unroll 1
  for (int j = 0; j < P.np; j++) {
    const int64_t x = pick<NC, R>(v, i, P.pred[j].mask);
    ok = ok && (present & P.pred[j].mask) && (x >= P.pred[j].lo) && (x <= P.pred[j].hi);
  }
  return ok;
}

// The columns an expression reads (a constant factor reads none).
__device__ __forceinline__ uint32_t expr_cols(const DExpr& E) {
  uint32_t m = 0;
#pragma unroll
  for (int f = 0; f < 3; f++)
    if (f < E.nf) m |= E.f[f].mask;
  return m;
}

// Exclusive prefix over the wave of a 32-bit value; *total gets the wave sum.
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

// Block-wide exclusive scan of one int64 per thread (blockDim a multiple of 64,
// at most 1024); returns the block total. Contains two barriers.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t* excl, int64_t* wave_sums) {
  const int lane = __lane_id(), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  int64_t s = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t y = __shfl_up(s, d, kWave);
    if (lane >= d) s += y;
  }
  if (lane == kWave - 1) wave_sums[wid] = s;
  __syncthreads();
  int64_t off = 0, total = 0;
  for (int w = 0; w < nw; w++) {
    int64_t t = wave_sums[w];
    off += w < wid ? t : 0;
    total += t;
  }
  __syncthreads();
  *excl = off + s - x;
  return total;
}

// Block-wide sum of one int64 per thread, result valid in every thread.
__device__ __forceinline__ int64_t block_sum(int64_t x, int64_t* wave_sums) {
  int64_t e;
  return block_excl_scan(x, &e, wave_sums);
}

// Block-wide sums of two int64 per thread, both valid in every thread.
// Contains two barriers.
__device__ __forceinline__ void block_sum2(int64_t* a, int64_t* b, int64_t* wave_vals) {
  const int lane = __lane_id(), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  int64_t x = *a, y = *b;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    x += __shfl_xor(x, d, kWave);
    y += __shfl_xor(y, d, kWave);
  }
  if (lane == 0) {
    wave_vals[2 * wid] = x;
    wave_vals[2 * wid + 1] = y;
  }
  __syncthreads();
  x = 0;
  y = 0;
  for (int w = 0; w < nw; w++) {
    x += wave_vals[2 * w];
    y += wave_vals[2 * w + 1];
  }
  __syncthreads();
  *a = x;
  *b = y;
}

// Block-wide sum and maximum of one int64 per thread, both valid in every
// thread. Contains two barriers.
__device__ __forceinline__ int64_t block_sum_max(int64_t x, int64_t* mx, int64_t* wave_vals) {
  const int lane = __lane_id(), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  int64_t s = x, m = x;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    s += __shfl_xor(s, d, kWave);
    const int64_t y = __shfl_xor(m, d, kWave);
    m = y > m ? y : m;
  }
  if (lane == 0) {
    wave_vals[2 * wid] = s;
    wave_vals[2 * wid + 1] = m;
  }
  __syncthreads();
  int64_t ts = 0, tm = wave_vals[1];
  for (int w = 0; w < nw; w++) {
    ts += wave_vals[2 * w];
    tm = wave_vals[2 * w + 1] > tm ? wave_vals[2 * w + 1] : tm;
  }
  __syncthreads();
  *mx = tm;
  return ts;
}

// Block-wide maximum of one int64 per thread, valid in every thread. Contains two barriers.
__device__ __forceinline__ int64_t block_max(int64_t x, int64_t* wave_vals) {
  const int lane = __lane_id(), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    int64_t y = __shfl_xor(x, d, kWave);
    x = y > x ? y : x;
  }
  if (lane == 0) wave_vals[wid] = x;
  __syncthreads();
  int64_t m = wave_vals[0];
  for (int w = 1; w < nw; w++) m = wave_vals[w] > m ? wave_vals[w] : m;
  __syncthreads();
  return m;
}

}  // namespace tq
