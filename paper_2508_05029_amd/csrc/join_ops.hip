// Open-addressing hash join: build (with the dimension filter fused in) and
// probe (aggregating matches in LDS, or materialising pairs in row order).
//
// Table layout: 256-byte header | int64 partial[2048] | uint16 tag[cap_max] |
// {int64 key, int64 payload}[cap_max]. Open addressing with linear probing over
// buckets of 8 slots: a key's home bucket is taken from the high bits of its
// 64-bit multiplicative hash, its tag from the low 16 bits (0 means empty).
// Inserts fill a bucket's free slots, then move to the next bucket; a probe
// reads the 8 tags of a bucket with one 16-byte load and stops at the first
// bucket that has an empty slot. The tags (2 bytes per slot) stay resident in
// L2, and the 16-byte slot is read only on a tag match, so at the load factors
// used here almost every probe costs one tag load (plus one slot load on a
// hit). Each lane walks the chains of its four rows in lockstep, so that four
// independent loads are in flight.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "groupby.h"
#include "table.h"

namespace tq {

constexpr int kBlock = 256;
constexpr int kChunk = kBlock * kRows;
constexpr int kPR = 2;  // rows per lane in the aggregating probe (fewer registers, more waves)

__host__ __device__ inline int log2cap_for(int64_t rows, double lf) {
  double need = ceil((double)rows / lf);
  int l = 6;
  while (l < 62 && (double)((int64_t)1 << l) < need) l++;
  return l;
}

__host__ __device__ inline size_t table_bytes_for(int64_t cap) {
  return kHeaderBytes + (size_t)kMaxPartBlocks * 8 + table_tag_bytes(cap) + (size_t)cap * 16;
}

static int64_t cap_max_for_bytes(size_t bytes) {
  int64_t cap = 0;
  for (int l = 6; l < 62; l++) {
    if (table_bytes_for((int64_t)1 << l) > bytes) break;
    cap = (int64_t)1 << l;
  }
  return cap;
}

struct Range {
  int64_t per;  // rows per block, a multiple of kChunk
  int nblk;
};

static Range split_rows(int64_t n, int max_blocks) {
  int64_t chunks = (n + kChunk - 1) / kChunk;
  int64_t nblk = std::min<int64_t>(std::max<int64_t>(chunks, 1), max_blocks);
  int64_t per = ((chunks + nblk - 1) / nblk) * kChunk;
  nblk = std::max<int64_t>(1, (n + per - 1) / per);
  return Range{per, (int)nblk};
}

static int stream_grid(int64_t n, int per_cu) {
  int64_t want = (n + kChunk - 1) / kChunk;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)device_cu_count() * per_cu));
}

__global__ void k_table_init(TableHeader* h, int64_t cap_max) {
  h->magic = kTableMagic;
  h->err = 0;
  h->cap_max = cap_max;
  h->log2cap = 6;
  h->skip = 0;
  h->n = 0;
  h->nblk = 0;
  h->flags = 0;
  h->lf = 0.5;
}

// ------------------------------------------------------------------ build

template <int NC>
__global__ __launch_bounds__(kBlock) void k_build_count(RowPlan P, int64_t n, int64_t per, TableHeader* h) {
  __shared__ int64_t ws[kBlock / kWave];
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  int64_t c = 0;
  for (int64_t r0 = lo + threadIdx.x * kRows; r0 < hi; r0 += kChunk) {
    int64_t v[NC][kRows];
    load_rows<NC>(P, r0, r0 + kRows <= hi, hi, v);
#pragma unroll
    for (int i = 0; i < kRows; i++) c += (r0 + i < hi) && eval_preds<NC>(P, v, i);
  }
  int64_t t = block_sum(c, ws);
  if (threadIdx.x == 0) table_partials(h)[blockIdx.x] = t;
}

// Fix the capacity from the row count (host-given, or the sum of the per-block
// counts) and clear the tags it uses.
__global__ __launch_bounds__(kBlock) void k_build_clear(TableHeader* h, int64_t cap_max, int64_t n_host, int nblk,
                                                        double lf, int skip, uint32_t flags) {
  __shared__ int64_t ws[kBlock / kWave];
  if (h->magic != kTableMagic) return;  // never initialised: the insert kernel does nothing either
  int64_t rows = n_host;
  if (n_host < 0) {
    int64_t c = 0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) c += table_partials(h)[b];
    rows = block_sum(c, ws);
  }
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
  const int64_t nb = ((int64_t)1 << l) >> kLog2Bucket;  // one 16-byte tag group per bucket
  const v4i32 z = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x)
    tags[i] = z;
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_build_insert(RowPlan P, const int64_t* keys, DCol payload, int64_t n,
                                                         TableHeader* h) {
  if (h->magic != kTableMagic) return;
  const int l = h->log2cap, skip = h->skip;
  if (h->n > ((int64_t)1 << l)) return;  // does not fit: TQ_EFULL is latched, nothing is inserted
  uint32_t* words = table_tags(h);
  v2i64* slots = reinterpret_cast<v2i64*>(table_slots(h, h->cap_max));
  const DCol kc = {keys, 8};
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    const bool full = r0 + kRows <= n;
    int64_t v[NC][kRows], k[kRows], pay[kRows];
    bool pend[kRows];
    load_rows<NC>(P, r0, full, n, v);
    load4(kc, r0, full, n, k);
    load4(payload, r0, full, n, pay);
#pragma unroll
    for (int i = 0; i < kRows; i++) pend[i] = (r0 + i < n) && eval_preds<NC>(P, v, i);
    table_insert<kRows>(words, slots, l, skip, pend, k, pay);
  }
}

// ------------------------------------------------------------------ probe

template <int MODE, int NC, int NE>
__global__ __launch_bounds__(kAggBlock, kAggBlocksPerCU) void k_probe_agg(const TableHeader* h, const int64_t* pkeys, int64_t n, RowPlan P,
                                                         AggTarget T) {
  extern __shared__ __align__(16) char smem[];
  if (h->magic != kTableMagic) return;
  if (!state_matches(T)) return;
  LdsAgg<MODE> agg;
  agg.init(T, smem);
  __syncthreads();
  Probe pr;
  pr.setup(h);
  const DCol kc = {pkeys, 8};
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kPR;
  // Software pipeline: the columns of the next rows are loaded while the
  // current rows walk the table.
  int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kPR;
  int64_t vn[NC][kPR], kn[kPR];
  if (r0 < n) {
    load_rows<NC>(P, r0, r0 + kPR <= n, n, vn);
    load4(kc, r0, r0 + kPR <= n, n, kn);
  }
  for (; r0 < n; r0 += step) {
    int64_t k[kPR], e[kPR][NE];
    bool ok[kPR];
#pragma unroll
    for (int i = 0; i < kPR; i++) {
      ok[i] = (r0 + i < n) && eval_preds<NC>(P, vn, i);
#pragma unroll
      for (int j = 0; j < NE; j++) e[i][j] = j < P.ne ? eval_expr<NC>(P.expr[j], vn, i) : 0;
      k[i] = kn[i];
    }
    const int64_t r1 = r0 + step;
    pr.walk(
        ok, k,
        [&](const bool (&hit)[kPR], const int64_t (&pay)[kPR]) {
#pragma unroll
          for (int i = 0; i < kPR; i++)
            if (hit[i]) agg.add(T, pay[i], e[i], P.ne);
        },
        [&] {
          if (r1 < n) {
            load_rows<NC>(P, r1, r1 + kPR <= n, n, vn);
            load4(kc, r1, r1 + kPR <= n, n, kn);
          }
        });
  }
  agg.flush(T);
}

// Match count of each block's contiguous row range (pairs mode, pass 1).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_probe_count(const TableHeader* h, const int64_t* pkeys, int64_t n,
                                                        int64_t per, RowPlan P, int64_t* cnt) {
  __shared__ int64_t ws[kBlock / kWave];
  if (h->magic != kTableMagic) return;
  Probe pr;
  pr.setup(h);
  const DCol kc = {pkeys, 8};
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  int64_t c = 0;
  for (int64_t r0 = lo + threadIdx.x * kRows; r0 < hi; r0 += kChunk) {
    const bool full = r0 + kRows <= hi;
    int64_t v[NC][kRows], k[kRows];
    bool ok[kRows];
    load_rows<NC>(P, r0, full, hi, v);
    load4(kc, r0, full, hi, k);
#pragma unroll
    for (int i = 0; i < kRows; i++) ok[i] = (r0 + i < hi) && eval_preds<NC>(P, v, i);
    pr.walk(ok, k, [&](const bool (&hit)[kRows], const int64_t (&)[kRows]) {
#pragma unroll
      for (int i = 0; i < kRows; i++) c += hit[i];
    });
  }
  int64_t t = block_sum(c, ws);
  if (threadIdx.x == 0) cnt[blockIdx.x] = t;
}

// Pairs mode, pass 2: write (row, payload) in probe-row order.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_probe_write(const TableHeader* h, const int64_t* pkeys, int64_t n,
                                                        int64_t per, RowPlan P, const int64_t* base, int64_t* out_row,
                                                        int64_t* out_pay, int64_t capacity) {
  __shared__ int64_t ws[kBlock / kWave];
  if (h->magic != kTableMagic) return;
  Probe pr;
  pr.setup(h);
  const DCol kc = {pkeys, 8};
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  int64_t w0 = base[blockIdx.x];
  for (int64_t c0 = lo; c0 < hi; c0 += kChunk) {  // uniform loop: every thread takes part in the scan
    const int64_t r0 = c0 + threadIdx.x * kRows;
    const bool full = r0 + kRows <= hi;
    int64_t v[NC][kRows], k[kRows];
    bool ok[kRows];
    if (r0 < hi) {
      load_rows<NC>(P, r0, full, hi, v);
      load4(kc, r0, full, hi, k);
    }
#pragma unroll
    for (int i = 0; i < kRows; i++) ok[i] = (r0 + i < hi) && eval_preds<NC>(P, v, i);
    int64_t mine = 0;
    pr.walk(ok, k, [&](const bool (&hit)[kRows], const int64_t (&)[kRows]) {
#pragma unroll
      for (int i = 0; i < kRows; i++) mine += hit[i];
    });
    int64_t excl;
    int64_t tot = block_excl_scan(mine, &excl, ws);
    int64_t w = w0 + excl;
    // a second walk emits the matches of each row in chain order
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      bool one[kRows];
      int64_t kk[kRows];
#pragma unroll
      for (int j = 0; j < kRows; j++) {
        one[j] = ok[j] && j == i;
        kk[j] = k[j];
      }
      pr.walk(one, kk, [&](const bool (&hit)[kRows], const int64_t (&pay)[kRows]) {
#pragma unroll
        for (int j = 0; j < kRows; j++) {
          if (hit[j]) {
            if (w < capacity) {
              out_row[w] = r0 + i;
              out_pay[w] = pay[j];
            }
            w++;
          }
        }
      });
    }
    w0 += tot;
  }
}

template <int D>
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t* cnt, int nblk, int64_t* total) {
  __shared__ int64_t ws[1024 / kWave];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nblk; b0 += 1024) {
    int b = b0 + threadIdx.x;
    int64_t x = b < nblk ? cnt[b] : 0, e;
    int64_t t = block_excl_scan(x, &e, ws);
    if (b < nblk) cnt[b] = carry + e;
    __syncthreads();
    if (threadIdx.x == 0) carry += t;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_zero1(int64_t* p) { *p = 0; }

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
  if (n < 0) return fail(TQ_EINVAL, "n < 0");
  if (n > 0 && (!d_keys || !payload.data)) return fail(TQ_EINVAL, "NULL keys or payload");
  if (((uintptr_t)d_keys & 15) || ((uintptr_t)payload.data & 15)) return fail(TQ_EINVAL, "keys/payload not 16-byte aligned");
  if (payload.type != TQ_U8 && payload.type != TQ_I32 && payload.type != TQ_I64) return fail(TQ_EINVAL, "payload type");
  int64_t cap_max = cap_max_for_bytes(bytes);
  if (cap_max == 0) return fail(TQ_EINVAL, "table buffer of %zu bytes is too small", bytes);
  RowPlan P;
  tq_status s = make_plan(&P, filt, nfilt, p, np, nullptr, 0, nullptr, n);
  if (s) return s;
  TableHeader* h = static_cast<TableHeader*>(d_table);
  int nblk = 0;
  if (np > 0 && n > 0) {
    Range R = split_rows(n, kMaxPartBlocks);
    nblk = R.nblk;
    TQ_DISPATCH_NC(nfilt, NC, hipLaunchKernelGGL(k_build_count<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, P, n, R.per, h));
    TQ_HIP(hipGetLastError());
  }
  int64_t clear_blocks = std::max<int64_t>(1, std::min<int64_t>(cap_max / 4 / kBlock, device_cu_count() * 4));
  hipLaunchKernelGGL(k_build_clear, dim3((int)clear_blocks), dim3(kBlock), 0, stream, h, cap_max,
                     np > 0 ? (int64_t)-1 : n, nblk, load_factor, skip, flags);
  TQ_HIP(hipGetLastError());
  if (n > 0) {
    DCol pc = {payload.data, payload.type};
    TQ_DISPATCH_NC(nfilt, NC, hipLaunchKernelGGL(k_build_insert<NC>, dim3(stream_grid(n, 8)), dim3(kBlock), 0, stream, P,
                                                 d_keys, pc, n, h));
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

tq_status tq_join_probe(const void* d_table, const int64_t* d_probe_keys, int64_t n, const tq_col* cols, int32_t ncol,
                        const tq_pred* p, int32_t np, int64_t* d_out_probe_row, int64_t* d_out_payload,
                        int64_t capacity, int64_t* d_out_count, const tq_agg* agg, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (n < 0) return fail(TQ_EINVAL, "n < 0");
  if (n > 0 && !d_probe_keys) return fail(TQ_EINVAL, "probe keys are NULL");
  if ((uintptr_t)d_probe_keys & 15) return fail(TQ_EINVAL, "probe keys not 16-byte aligned");
  RowPlan P;
  tq_status s = make_plan(&P, cols, ncol, p, np, agg ? agg->sums : nullptr, agg ? agg->nsum : 0, nullptr, n);
  if (s) return s;
  const TableHeader* h = static_cast<const TableHeader*>(d_table);
  if (agg) {
    AggTarget T{};
    AggMode mode;
    size_t lds = 0;
    if ((s = make_target(agg->d_state, agg->domain, agg->nsum, &T, &mode, &lds))) return s;
    if (d_out_count) return fail(TQ_EINVAL, "the fused group-by counts matches in its COUNT column; pass d_out_count = NULL");
    if (n == 0) return TQ_OK;
    dim3 grid(agg_grid(n)), block(kAggBlock);
    TQ_DISPATCH_AGG(mode, ncol, agg->nsum, M, NC, NE,
                    hipLaunchKernelGGL((k_probe_agg<M, NC, NE>), grid, block, lds, stream, h, d_probe_keys, n, P, T));
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  if (!d_out_count) return fail(TQ_EINVAL, "d_out_count is NULL");
  if (capacity < 0 || (capacity > 0 && (!d_out_probe_row || !d_out_payload))) return fail(TQ_EINVAL, "bad pair outputs");
  if (n == 0) {
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, stream, d_out_count);
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  Range R = split_rows(n, kMaxPartBlocks);
  // the per-block counts live in the table's partial area: materialising probes of one table must not overlap
  int64_t* cnt = table_partials(const_cast<void*>(d_table));
  TQ_DISPATCH_NC(ncol, NC, hipLaunchKernelGGL(k_probe_count<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, h, d_probe_keys, n,
                                              R.per, P, cnt));
  hipLaunchKernelGGL(k_scan_blocks<0>, dim3(1), dim3(1024), 0, stream, cnt, R.nblk, d_out_count);
  TQ_DISPATCH_NC(ncol, NC, hipLaunchKernelGGL(k_probe_write<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, h, d_probe_keys, n,
                                              R.per, P, cnt, d_out_probe_row, d_out_payload, capacity));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
