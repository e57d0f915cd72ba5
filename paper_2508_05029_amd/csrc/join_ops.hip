// Open-addressing hash join: build (with the dimension filter fused in) and
// probe (materialising pairs, or aggregating matches in LDS).
//
// Table layout: 256-byte header | uint32 tag[cap_max] | {int64 key, int64 payload}[cap_max].
// A slot is empty iff its tag is 0; the tag is the low 32 bits of the hash
// (0 mapped to 1). A probe walks tags, which stay resident in L2 (4 bytes per
// slot), and reads the 16-byte slot only when the tag matches, so most misses
// never touch the slot array.
#include <math.h>

#include "common.h"
#include "groupby.h"

namespace tq {

constexpr int kBlock = 256;

static int blocks_for(int64_t n, int per_cu) {
  int64_t want = (n + (int64_t)kBlock * kRows - 1) / ((int64_t)kBlock * kRows);
  int64_t cap = (int64_t)device_cu_count() * per_cu;
  if (want < 1) want = 1;
  return (int)(want < cap ? want : cap);
}

__host__ __device__ inline int log2cap_for(int64_t rows, double lf) {
  double need = ceil((double)rows / lf);
  int l = 6;
  while (l < 62 && (double)((int64_t)1 << l) < need) l++;
  return l;
}

__host__ __device__ inline size_t table_bytes_for(int64_t cap) {
  return kHeaderBytes + (((size_t)cap * 4 + 255) & ~(size_t)255) + (size_t)cap * 16;
}

static int64_t cap_max_for_bytes(size_t bytes) {
  int64_t cap = 0;
  for (int l = 6; l < 62; l++) {
    if (table_bytes_for((int64_t)1 << l) > bytes) break;
    cap = (int64_t)1 << l;
  }
  return cap;
}

__global__ void k_table_init(TableHeader* h, int64_t cap_max) {
  h->magic = kTableMagic;
  h->err = 0;
  h->cap_max = cap_max;
  h->log2cap = 6;
  h->skip = 0;
  h->n = 0;
  h->n_acc = 0;
  h->ticket = 0;
  h->flags = 0;
  h->lf = 0.5;
}

// Count the build rows that pass the filter; the last workgroup publishes the total.
__global__ __launch_bounds__(kBlock) void k_build_count(RowPlan P, int64_t n, TableHeader* h) {
  __shared__ int64_t part[kBlock / kWave];
  int64_t cnt = 0;
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    bool full = r0 + kRows <= n;
    int64_t v[TQ_MAX_COLS][kRows];
#pragma unroll
    for (int c = 0; c < TQ_MAX_COLS; c++)
      if (c < P.ncol) load4(P.col[c], r0, full, n, v[c]);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      cnt += (r0 + i < n) && eval_preds(P, vals);
    }
  }
  for (int d = 32; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, kWave);
  if (__lane_id() == 0) part[threadIdx.x / kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kBlock / kWave; w++) t += part[w];
    atomicAdd(reinterpret_cast<unsigned long long*>(&h->n_acc), (unsigned long long)t);
    __threadfence();
    uint32_t ticket = atomicAdd(&h->ticket, 1u);
    if (ticket == gridDim.x - 1) {
      __threadfence();
      int64_t total = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&h->n_acc), 0ull);
      h->n = total;
      h->n_acc = 0;
      h->ticket = 0;
    }
  }
}

// Fix the capacity from the row count and clear the tags it uses.
__global__ __launch_bounds__(kBlock) void k_build_clear(TableHeader* h, int64_t cap_max, int64_t n_host, double lf,
                                                        int skip, uint32_t flags) {
  if (h->magic != kTableMagic) return;  // never initialised: the insert kernel does nothing either
  const int64_t rows = n_host >= 0 ? n_host : h->n;
  int l = log2cap_for(rows, lf);
  bool full = ((int64_t)1 << l) > cap_max;
  if (full) {
    l = 6;
    while (((int64_t)1 << (l + 1)) <= cap_max) l++;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->cap_max = cap_max;
    h->n = rows;
    h->log2cap = l;
    h->skip = skip;
    h->flags = flags;
    h->lf = lf;
    if (full) latch_error(&h->err, TQ_EFULL);
  }
  v4i32* tags = reinterpret_cast<v4i32*>(table_tags(h));
  const int64_t n16 = ((int64_t)1 << l) / 4;
  const v4i32 z = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    tags[i] = z;
}

__global__ __launch_bounds__(kBlock) void k_build_insert(RowPlan P, const int64_t* keys, DCol payload, int64_t n,
                                                         TableHeader* h) {
  if (h->magic != kTableMagic) return;
  const int l = h->log2cap, skip = h->skip;
  const int64_t cap = (int64_t)1 << l, mask = cap - 1;
  if (h->n > cap) return;  // does not fit: TQ_EFULL is latched, nothing is inserted
  uint32_t* tags = table_tags(h);
  v2i64* slots = reinterpret_cast<v2i64*>(table_slots(h, h->cap_max));
  const DCol kc = {keys, 8};
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    bool full = r0 + kRows <= n;
    int64_t v[TQ_MAX_COLS][kRows], k[kRows], pay[kRows];
#pragma unroll
    for (int c = 0; c < TQ_MAX_COLS; c++)
      if (c < P.ncol) load4(P.col[c], r0, full, n, v[c]);
    load4(kc, r0, full, n, k);
    load4(payload, r0, full, n, pay);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      if (r0 + i >= n) break;
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      if (!eval_preds(P, vals)) continue;
      uint64_t hh = mulhash(k[i]);
      int64_t s = (int64_t)slot_of(hh, skip, l);
      uint32_t tag = hash_tag(hh);
      for (int64_t t = 0; t < cap; t++) {
        if (atomicCAS(&tags[s], 0u, tag) == 0u) {
          v2i64 kv = {k[i], pay[i]};
          slots[s] = kv;
          break;
        }
        s = (s + 1) & mask;
      }
    }
  }
}

// ------------------------------------------------------------------ probe

constexpr int kPairs = 3;  // materialise (row, payload) pairs instead of aggregating

struct PairOut {
  int64_t* row;
  int64_t* payload;
  int64_t capacity;
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_probe(const TableHeader* h, const int64_t* pkeys, int64_t n, RowPlan P,
                                                  PairOut out, unsigned long long* count, AggTarget T) {
  extern __shared__ __align__(16) char smem[];
  if (h->magic != kTableMagic) return;
  if (MODE != kPairs && !state_matches(T)) return;
  LdsAgg<MODE == kPairs ? kGlobal : MODE> agg;
  if (MODE != kPairs) agg.init(T, smem);
  __syncthreads();

  const int l = h->log2cap, skip = h->skip;
  const bool unique = (h->flags & TQ_UNIQUE_KEYS) != 0;
  const int64_t cap = (int64_t)1 << l, mask = cap - 1;
  const uint32_t* tags = table_tags(const_cast<TableHeader*>(h));
  const v2i64* slots = reinterpret_cast<const v2i64*>(table_slots(const_cast<TableHeader*>(h), h->cap_max));
  const DCol kc = {pkeys, 8};
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  uint32_t matches = 0;

  // Pairs mode runs whole waves through the loop so that the wave scan sees every lane.
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows;
       MODE == kPairs ? (r0 - (int64_t)threadIdx.x * kRows < n) : (r0 < n); r0 += step) {
    const bool any = r0 < n;
    bool full = r0 + kRows <= n;
    int64_t v[TQ_MAX_COLS][kRows], k[kRows];
#pragma unroll
    for (int c = 0; c < TQ_MAX_COLS; c++)
      if (c < P.ncol && any) load4(P.col[c], r0, full, n, v[c]);
    if (any) load4(kc, r0, full, n, k);
    bool ok[kRows];
    int64_t s[kRows];
    uint32_t tg[kRows], t0[kRows];
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      ok[i] = any && (r0 + i < n) && eval_preds(P, vals);
      uint64_t hh = mulhash(k[i]);
      s[i] = (int64_t)slot_of(hh, skip, l);
      tg[i] = hash_tag(hh);
    }
    // issue the first tag load of every row before walking any chain
#pragma unroll
    for (int i = 0; i < kRows; i++) t0[i] = ok[i] ? tags[s[i]] : 0u;

    if (MODE == kPairs) {
      uint32_t mine = 0;
#pragma unroll
      for (int i = 0; i < kRows; i++) {
        int64_t si = s[i];
        uint32_t t = t0[i];
        for (int64_t it = 0; t != 0 && it < cap; it++) {
          if (t == tg[i] && slots[si].x == k[i]) {
            mine++;
            if (unique) break;
          }
          si = (si + 1) & mask;
          t = tags[si];
        }
      }
      uint32_t total;
      uint32_t pre = wave_excl_scan(mine, &total);
      unsigned long long base = 0;
      if (__lane_id() == kWave - 1 && total) base = atomicAdd(count, (unsigned long long)total);
      base = __shfl(base, kWave - 1, kWave);
      int64_t w = (int64_t)base + pre;
#pragma unroll
      for (int i = 0; i < kRows; i++) {
        int64_t si = s[i];
        uint32_t t = t0[i];
        for (int64_t it = 0; t != 0 && it < cap; it++) {
          if (t == tg[i]) {
            v2i64 kv = slots[si];
            if (kv.x == k[i]) {
              if (w < out.capacity) {
                out.row[w] = r0 + i;
                out.payload[w] = kv.y;
              }
              w++;
              if (unique) break;
            }
          }
          si = (si + 1) & mask;
          t = tags[si];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < kRows; i++) {
        int64_t si = s[i];
        uint32_t t = t0[i];
        for (int64_t it = 0; t != 0 && it < cap; it++) {
          if (t == tg[i]) {
            v2i64 kv = slots[si];
            if (kv.x == k[i]) {
              int64_t vals[TQ_MAX_COLS], e[TQ_MAX_SUMS];
#pragma unroll
              for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
#pragma unroll
              for (int j = 0; j < TQ_MAX_SUMS; j++)
                if (j < P.ne) e[j] = eval_expr(P.expr[j], vals);
              agg.add(T, kv.y, e, P.ne);
              matches++;
              if (unique) break;
            }
          }
          si = (si + 1) & mask;
          t = tags[si];
        }
      }
    }
  }
  if (MODE != kPairs) {
    agg.flush(T);
    if (count) {
      for (int d = 32; d > 0; d >>= 1) matches += __shfl_xor(matches, d, kWave);
      if (__lane_id() == 0 && matches) atomicAdd(count, (unsigned long long)matches);
    }
  }
}

__global__ void k_zero1(int64_t* p) { *p = 0; }

tq_status make_target(void* d_state, int64_t domain, int32_t nsum, AggTarget* T, AggMode* mode, size_t* lds);

}  // namespace tq

using namespace tq;

extern "C" {

size_t tq_join_table_bytes(int64_t n_build_max, double load_factor) {
  if (n_build_max < 0 || !(load_factor > 0.0 && load_factor <= 0.9)) return 0;
  return table_bytes_for((int64_t)1 << log2cap_for(n_build_max, load_factor));
}

tq_status tq_join_table_init(void* d_table, size_t bytes, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  int64_t cap_max = cap_max_for_bytes(bytes);
  if (cap_max == 0) return fail(TQ_EINVAL, "table buffer of %zu bytes is too small", bytes);
  hipLaunchKernelGGL(k_table_init, dim3(1), dim3(1), 0, stream, static_cast<TableHeader*>(d_table), cap_max);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_join_build(void* d_table, size_t bytes, const int64_t* d_keys, tq_col payload, int64_t n,
                        const tq_col* filt, int32_t nfilt, const tq_pred* p, int32_t np, double load_factor,
                        int32_t skip, uint32_t flags, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (!(load_factor > 0.0 && load_factor <= 0.9)) return fail(TQ_EINVAL, "load factor %g outside (0, 0.9]", load_factor);
  if (skip < 0 || skip > 32) return fail(TQ_EINVAL, "skip %d outside [0, 32]", skip);
  if (n > 0 && (!d_keys || !payload.data)) return fail(TQ_EINVAL, "NULL keys or payload");
  if (((uintptr_t)d_keys & 15) || ((uintptr_t)payload.data & 15)) return fail(TQ_EINVAL, "keys/payload not 16-byte aligned");
  if (payload.type != TQ_U8 && payload.type != TQ_I32 && payload.type != TQ_I64) return fail(TQ_EINVAL, "payload type");
  int64_t cap_max = cap_max_for_bytes(bytes);
  if (cap_max == 0) return fail(TQ_EINVAL, "table buffer of %zu bytes is too small", bytes);
  RowPlan P;
  tq_status s = make_plan(&P, filt, nfilt, p, np, nullptr, 0, nullptr, n);
  if (s) return s;
  TableHeader* h = static_cast<TableHeader*>(d_table);
  int grid = blocks_for(n, 8);
  if (np > 0 && n > 0) {
    hipLaunchKernelGGL(k_build_count, dim3(grid), dim3(kBlock), 0, stream, P, n, h);
    TQ_HIP(hipGetLastError());
  }
  int64_t clear_blocks = std::max<int64_t>(1, std::min<int64_t>(cap_max / 4 / kBlock, device_cu_count() * 4));
  hipLaunchKernelGGL(k_build_clear, dim3((int)clear_blocks), dim3(kBlock), 0, stream, h, cap_max,
                     np > 0 ? (int64_t)-1 : n, load_factor, skip, flags);
  TQ_HIP(hipGetLastError());
  if (n > 0) {
    DCol pc = {payload.data, payload.type};
    hipLaunchKernelGGL(k_build_insert, dim3(grid), dim3(kBlock), 0, stream, P, d_keys, pc, n, h);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

tq_status tq_join_probe(const void* d_table, const int64_t* d_probe_keys, int64_t n, const tq_col* cols, int32_t ncol,
                        const tq_pred* p, int32_t np, int64_t* d_out_probe_row, int64_t* d_out_payload,
                        int64_t capacity, int64_t* d_out_count, const tq_agg* agg, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (n > 0 && !d_probe_keys) return fail(TQ_EINVAL, "probe keys are NULL");
  if ((uintptr_t)d_probe_keys & 15) return fail(TQ_EINVAL, "probe keys not 16-byte aligned");
  RowPlan P;
  tq_status s = make_plan(&P, cols, ncol, p, np, agg ? agg->sums : nullptr, agg ? agg->nsum : 0, nullptr, n);
  if (s) return s;
  const TableHeader* h = static_cast<const TableHeader*>(d_table);
  AggTarget T{};
  AggMode mode = kGlobal;
  size_t lds = 0;
  if (agg) {
    if ((s = make_target(agg->d_state, agg->domain, agg->nsum, &T, &mode, &lds))) return s;
  } else {
    if (!d_out_count) return fail(TQ_EINVAL, "d_out_count is NULL");
    if (capacity < 0 || (capacity > 0 && (!d_out_probe_row || !d_out_payload)))
      return fail(TQ_EINVAL, "bad pair outputs");
  }
  if (d_out_count) {
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, stream, d_out_count);
    TQ_HIP(hipGetLastError());
  }
  if (n == 0) return TQ_OK;
  PairOut out = {d_out_probe_row, d_out_payload, capacity};
  auto* cnt = reinterpret_cast<unsigned long long*>(d_out_count);
  dim3 grid(blocks_for(n, agg ? 4 : 8)), block(kBlock);
  if (!agg) hipLaunchKernelGGL(k_probe<kPairs>, grid, block, 0, stream, h, d_probe_keys, n, P, out, cnt, T);
  else if (mode == kDense) hipLaunchKernelGGL(k_probe<kDense>, grid, block, lds, stream, h, d_probe_keys, n, P, out, cnt, T);
  else if (mode == kHash) hipLaunchKernelGGL(k_probe<kHash>, grid, block, lds, stream, h, d_probe_keys, n, P, out, cnt, T);
  else hipLaunchKernelGGL(k_probe<kGlobal>, grid, block, 0, stream, h, d_probe_keys, n, P, out, cnt, T);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
