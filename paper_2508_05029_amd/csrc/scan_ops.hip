// Filter / project (stable compaction), group-by accumulation and
// finalization, and the two measurement kernels (streaming read, fill).
#include <string.h>

#include <algorithm>

#include "common.h"
#include "groupby.h"

namespace tq {

constexpr int kBlock = 256;
constexpr int kChunk = kBlock * kRows;  // rows per block step of the compaction kernels
constexpr int kMaxScanBlocks = 2048;

__global__ void k_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Exclusive scan of up to kMaxScanBlocks per-block counts in one workgroup;
// writes the total to *total (if not NULL).
__global__ __launch_bounds__(1024) void k_scan_counts(int64_t* cnt, int nblk, int64_t* total) {
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

// ------------------------------------------------------------ filter/project

struct OutPtrs {
  int64_t* p[TQ_MAX_SUMS];
};

struct Range {
  int64_t per;  // rows per block, a multiple of kChunk
  int nblk;
};

static Range split_rows(int64_t n) {
  int64_t chunks = (n + kChunk - 1) / kChunk;
  int64_t nblk = std::min<int64_t>(std::max<int64_t>(chunks, 1), kMaxScanBlocks);
  int64_t per = ((chunks + nblk - 1) / nblk) * kChunk;
  nblk = std::max<int64_t>(1, (n + per - 1) / per);
  return Range{per, (int)nblk};
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_fp_count(RowPlan P, int64_t n, int64_t per, int64_t* cnt) {
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
  if (threadIdx.x == 0) cnt[blockIdx.x] = t;
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_fp_write(RowPlan P, int64_t n, int64_t per, const int64_t* base,
                                                     OutPtrs out, int64_t* sel) {
  __shared__ int64_t ws[kBlock / kWave];
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  int64_t w0 = base[blockIdx.x];
  for (int64_t c0 = lo; c0 < hi; c0 += kChunk) {  // uniform loop: every thread takes part in the scan
    const int64_t r0 = c0 + threadIdx.x * kRows;
    int64_t v[NC][kRows];
    bool ok[kRows];
    int64_t mine = 0;
    if (r0 < hi) load_rows<NC>(P, r0, r0 + kRows <= hi, hi, v);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      ok[i] = (r0 + i < hi) && eval_preds<NC>(P, v, i);
      mine += ok[i];
    }
    int64_t excl;
    int64_t tot = block_excl_scan(mine, &excl, ws);
    int64_t w = w0 + excl;
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      if (!ok[i]) continue;
#pragma unroll
      for (int e = 0; e < TQ_MAX_SUMS; e++)
        if (e < P.ne) out.p[e][w] = eval_expr<NC>(P.expr[e], v, i);
      if (sel) sel[w] = r0 + i;
      w++;
    }
    w0 += tot;
  }
}

// ------------------------------------------------------------ group-by

int agg_grid(int64_t n) {
  int64_t want = (n + (int64_t)kAggBlock * kRows - 1) / ((int64_t)kAggBlock * kRows);
  int64_t cap = std::min<int64_t>(kAggRows, kAggBlocksPerCU * (int64_t)device_cu_count());
  return (int)std::max<int64_t>(1, std::min(want, cap));
}

// NULLS: a nullable state (T.nullable) and columns that may carry validity
// bitmaps: a predicate over NULL drops the row, a NULL key goes to the NULL
// group (key T.udomain), and a sum whose expression reads a NULL value skips
// the row (entries 1 + 2e and 2 + 2e hold SUM_e and COUNT_e).
template <int MODE, int NC, bool NULLS>
__global__ __launch_bounds__(kAggBlock, kAggBlocksPerCU) void k_groupby(RowPlan P, int64_t n, AggTarget T) {
  extern __shared__ __align__(16) char smem[];
  if (!state_matches(T)) return;
  LdsAgg<MODE> agg;
  agg.init(T, smem);
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  const uint32_t key_cols = P.key_mask[0] | P.key_mask[1];
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    int64_t v[NC][kRows];
    load_rows<NC>(P, r0, r0 + kRows <= n, n, v);
    bool ok[kRows], lds[kRows];
    unsigned long long* at[kRows];
    uint32_t present[kRows];
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      if constexpr (NULLS) {
        present[i] = r0 + i < n ? row_present<NC>(P, r0 + i) : 0u;
        int64_t key = eval_key<NC>(P, v, i);
        // a NULL key is the NULL group; a present key outside [0, udomain) is an error (-1)
        key = (present[i] & key_cols) != key_cols ? T.udomain : ((uint64_t)key < (uint64_t)T.udomain ? key : -1);
        ok[i] = r0 + i < n && eval_preds_present<NC>(P, v, i, present[i]) && agg.count(T, key, &at[i], &lds[i]);
      } else {
        present[i] = ~0u;
        ok[i] = r0 + i < n && eval_preds<NC>(P, v, i) && agg.count(T, eval_key<NC>(P, v, i), &at[i], &lds[i]);
      }
    }
    // sums one at a time over the tile's rows, so that only one sum's plan
    // constants are live (all of them at once spill into vector lanes)
#pragma unroll 1
    for (int e = 0; e < P.ne; e++) {
      const DExpr E = P.expr[e];
      if constexpr (NULLS) {
        const uint32_t ec = expr_cols(E);
#pragma unroll
        for (int i = 0; i < kRows; i++) {
          if (ok[i] && (present[i] & ec) == ec) {
            const int64_t x = eval_expr<NC>(E, v, i);
            if (lds[i]) {
              atomicAdd(at[i] + 1 + 2 * e, (unsigned long long)x);
              atomicAdd(at[i] + 2 + 2 * e, 1ull);
            } else {
              global_add(at[i] + 1 + 2 * e, x);
              global_add(at[i] + 2 + 2 * e, 1);
            }
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < kRows; i++) {
          if (ok[i]) {
            const int64_t x = eval_expr<NC>(E, v, i);
            if (lds[i]) atomicAdd(at[i] + 1 + e, (unsigned long long)x);
            else global_add(at[i] + 1 + e, x);
          }
        }
      }
    }
  }
  agg.flush(T);
}

__global__ void k_state_init(StateHeader* h, int64_t domain, int32_t nsum, int32_t rows, int64_t entries,
                             int32_t nullable) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->magic = kStateMagic;
    h->err = 0;
    h->domain = domain;
    h->nsum = nsum;
    h->rows = rows;
    h->used = 0;
    h->nullable = nullable;
  }
  int64_t* d = state_data(h);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = 0;
}

// One workgroup: fold the private rows (if any), keep COUNT > 0, emit in key order.
constexpr int kFinBlock = 1024;

// With `reset`, every partial read is zeroed right after (the same thread, so
// the store follows its load) and the count of used private rows goes to 0:
// the state is then as tq_groupby_init leaves it, its error word aside.
// With a nullable state, sum j of a group is SUM_j over COUNT_j rows (entries
// 1 + 2j and 2 + 2j): d_sums gets SUM_j, d_nonnull COUNT_j, d_avg SUM_j /
// COUNT_j (0 when COUNT_j is 0), and the last group is the NULL key's.
__global__ __launch_bounds__(kFinBlock) void k_finalize(StateHeader* h, int64_t* keys, int64_t* count,
                                                        int64_t* sums, double* avg, int64_t* ngroups, int reset,
                                                        int64_t* nonnull) {
  __shared__ uint32_t wave_tot[kFinBlock / kWave];
  __shared__ int64_t fold[kPrivateRowsMaxEntries];
  __shared__ int64_t base_s;
  if (h->magic != kStateMagic) return;
  if ((h->nullable != 0) != (nonnull != nullptr)) {  // the finalize call does not fit the state
    if (threadIdx.x == 0) {
      latch_error(&h->err, TQ_EINVAL);
      *ngroups = 0;
    }
    return;
  }
  const int64_t domain = h->domain;
  const int stride = 1 + h->nsum, rows = h->rows;
  const bool nl = h->nullable != 0;
  const int nsum = nl ? h->nsum / 2 : h->nsum;  // the caller's sums
  int64_t* d = state_data(h);
  const int entries = (int)(domain * stride);
  if (rows > 1) {
    for (int e = threadIdx.x; e < entries; e += kFinBlock) fold[e] = 0;
    __syncthreads();
    // thread t < lim owns entry t % entries and every per-th used row from
    // t / entries: it sums them in a register (eight independent loads in
    // flight), then one LDS atomic per thread folds the sums
    const int per = kFinBlock / entries, lim = per * entries;
    const int nrow = (int)min<int64_t>(h->used, rows);
    if ((int)threadIdx.x < lim) {
      const int e = threadIdx.x % entries;
      uint64_t acc = 0;
      for (int r = threadIdx.x / entries; r < nrow; r += 8 * per) {
        uint64_t x[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int rr = r + u * per;
          x[u] = rr < nrow ? (uint64_t)d[(int64_t)rr * entries + e] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) acc += x[u];
        if (reset) {
#pragma unroll
          for (int u = 0; u < 8; u++) {
            const int rr = r + u * per;
            if (rr < nrow) d[(int64_t)rr * entries + e] = 0;
          }
        }
      }
      if (acc) atomicAdd(reinterpret_cast<unsigned long long*>(&fold[e]), (unsigned long long)acc);
    }
  }
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  const int wid = threadIdx.x / kWave, lane = __lane_id();
  for (int64_t k0 = 0; k0 < domain; k0 += kFinBlock) {
    int64_t k = k0 + threadIdx.x;
    int64_t e[1 + TQ_MAX_SUMS];
    bool live = false;
    if (k < domain) {
#pragma unroll
      for (int j = 0; j < 1 + TQ_MAX_SUMS; j++)
        if (j < stride) e[j] = rows > 1 ? fold[k * stride + j] : d[k * stride + j];
      if (reset && rows == 1) {
#pragma unroll
        for (int j = 0; j < 1 + TQ_MAX_SUMS; j++)
          if (j < stride) d[k * stride + j] = 0;
      }
      live = e[0] != 0;
    }
    uint64_t m = __ballot(live);
    uint32_t pre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wid] = __popcll(m);
    __syncthreads();
    int64_t off = base_s;
    for (int w = 0; w < wid; w++) off += wave_tot[w];
    if (live) {
      int64_t g = off + pre;
      keys[g] = k;
      count[g] = e[0];
      if (nl) {
#pragma unroll
        for (int j = 0; j < kMaxNullableSums; j++) {
          if (j < nsum) {
            const int64_t sj = e[1 + 2 * j], cj = e[2 + 2 * j];
            sums[g * nsum + j] = cj ? sj : 0;
            nonnull[g * nsum + j] = cj;
            if (avg) avg[g * nsum + j] = cj ? (double)sj / (double)cj : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < TQ_MAX_SUMS; j++) {
          if (j < nsum) {
            sums[g * nsum + j] = e[1 + j];
            if (avg) avg[g * nsum + j] = (double)e[1 + j] / (double)e[0];
          }
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < kFinBlock / kWave; w++) t += wave_tot[w];
      base_s += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ngroups = base_s;
    if (reset) h->used = 0;  // (read above by every thread, before the loop's barriers)
  }
}

// ------------------------------------------------------------ measurement

__global__ __launch_bounds__(kBlock) void k_read_peak(const v2i64* src, int64_t n16, int64_t* part) {
  __shared__ int64_t ws[kBlock / kWave];
  long long acc = 0;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * step < n16; i += 4 * step) {
    v2i64 a = ntload(src + i), b = ntload(src + i + step), c = ntload(src + i + 2 * step), e = ntload(src + i + 3 * step);
    acc += a.x + a.y + b.x + b.y + c.x + c.y + e.x + e.y;
  }
  for (; i < n16; i += step) {
    v2i64 a = ntload(src + i);
    acc += a.x + a.y;
  }
  int64_t t = block_sum(acc, ws);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_fill(v4i32* dst, int64_t n16, uint32_t pattern) {
  v4i32 v = {(int)pattern, (int)pattern, (int)pattern, (int)pattern};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(v, dst + i);
}

tq_status make_target(void* d_state, int64_t domain, int32_t nsum, AggTarget* T, AggMode* mode, size_t* lds,
                      bool nullable) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (domain <= 0 || domain > ((int64_t)1 << 31)) return fail(TQ_EINVAL, "domain %lld outside [1, 2^31]", (long long)domain);
  const int max_sums = nullable ? kMaxNullableSums : TQ_MAX_SUMS;
  if (nsum < 0 || nsum > max_sums) return fail(TQ_EINVAL, "nsum %d outside [0, %d]", nsum, max_sums);
  T->hdr = static_cast<const StateHeader*>(d_state);
  T->data = state_data(d_state);
  T->err = &static_cast<StateHeader*>(d_state)->err;
  T->nullable = nullable ? 1 : 0;
  T->udomain = domain;
  T->domain = nullable ? domain + 1 : domain;  // the NULL group follows the keys
  T->stride = nullable ? 1 + 2 * nsum : 1 + nsum;
  T->rows = state_rows(T->domain, T->stride);
  *mode = agg_mode(T->domain, T->stride, &T->log2hcap, lds);
  return TQ_OK;
}

}  // namespace tq

using namespace tq;

extern "C" {

size_t tq_filter_project_scratch_bytes(int64_t nrows) {
  if (nrows < 0) return 0;
  return (size_t)kMaxScanBlocks * 8;
}

tq_status tq_filter_project(const tq_col* in, int32_t ncol, int64_t nrows, const tq_pred* p, int32_t np,
                            const tq_expr* e, int32_t ne, int64_t* const* d_out, int64_t* d_sel, int64_t* d_out_rows,
                            void* d_scratch, size_t scratch_bytes, hipStream_t stream) {
  RowPlan P;
  tq_status s = make_plan(&P, in, ncol, p, np, e, ne, nullptr, nrows);
  if (s) return s;
  if (!d_out_rows) return fail(TQ_EINVAL, "d_out_rows is NULL");
  if (!d_scratch || scratch_bytes < tq_filter_project_scratch_bytes(nrows))
    return fail(TQ_EINVAL, "scratch needs %zu bytes", tq_filter_project_scratch_bytes(nrows));
  OutPtrs out{};
  for (int j = 0; j < ne; j++) {
    if (!d_out || !d_out[j]) return fail(TQ_EINVAL, "output %d is NULL", j);
    out.p[j] = d_out[j];
  }
  if (nrows == 0) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, stream, d_out_rows, (int64_t)1);
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  Range R = split_rows(nrows);
  int64_t* cnt = static_cast<int64_t*>(d_scratch);
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_fp_count<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, P, nrows, R.per, cnt));
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, stream, cnt, R.nblk, d_out_rows);
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_fp_write<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, P, nrows, R.per, cnt, out, d_sel));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

size_t tq_groupby_state_bytes(int64_t domain, int32_t nsum) {
  if (domain <= 0 || domain > ((int64_t)1 << 31) || nsum < 0 || nsum > TQ_MAX_SUMS) return 0;
  int stride = 1 + nsum;
  return kHeaderBytes + (size_t)state_rows(domain, stride) * (size_t)domain * stride * 8;
}

static tq_status init_state(void* d_state, size_t bytes, int64_t domain, int32_t nsum, bool nullable,
                            hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "state is NULL");
  if (domain <= 0 || domain > (int64_t)1 << 31) return fail(TQ_EINVAL, "domain %lld outside [1, 2^31]", (long long)domain);
  const int max_sums = nullable ? kMaxNullableSums : TQ_MAX_SUMS;
  if (nsum < 0 || nsum > max_sums) return fail(TQ_EINVAL, "nsum %d outside [0, %d]", nsum, max_sums);
  size_t need = nullable ? tq_groupby_state_bytes_nullable(domain, nsum) : tq_groupby_state_bytes(domain, nsum);
  if (bytes < need) return fail(TQ_EINVAL, "state buffer has %zu bytes, needs %zu", bytes, need);
  const int64_t groups = nullable ? domain + 1 : domain;  // the NULL group follows the keys
  const int32_t entry_sums = nullable ? 2 * nsum : nsum;   // SUM_j and COUNT_j per sum
  int stride = 1 + entry_sums;
  int rows = state_rows(groups, stride);
  int64_t entries = (int64_t)rows * groups * stride;
  int blocks = (int)std::min<int64_t>((entries + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_state_init, dim3(blocks), dim3(kBlock), 0, stream, static_cast<StateHeader*>(d_state), groups,
                     entry_sums, rows, entries, nullable ? 1 : 0);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_groupby_init(void* d_state, size_t bytes, int64_t domain, int32_t nsum, hipStream_t stream) {
  return init_state(d_state, bytes, domain, nsum, false, stream);
}

size_t tq_groupby_state_bytes_nullable(int64_t domain, int32_t nsum) {
  if (domain <= 0 || domain >= ((int64_t)1 << 31) || nsum < 0 || nsum > kMaxNullableSums) return 0;
  const int stride = 1 + 2 * nsum;
  return kHeaderBytes + (size_t)state_rows(domain + 1, stride) * (size_t)(domain + 1) * stride * 8;
}

tq_status tq_groupby_init_nullable(void* d_state, size_t bytes, int64_t domain, int32_t nsum, hipStream_t stream) {
  return init_state(d_state, bytes, domain, nsum, true, stream);
}

static tq_status groupby_agg(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                             const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                             bool nullable, hipStream_t stream) {
  if (!key) return fail(TQ_EINVAL, "group key is NULL");
  if (nullable && key->ncol != 1) return fail(TQ_EINVAL, "a group key that may be NULL has one column");
  RowPlan P;
  tq_status s = make_plan(&P, in, ncol, p, np, sums, nsum, key, nrows, nullable);
  if (s) return s;
  AggTarget T;
  AggMode mode;
  size_t lds;
  if ((s = make_target(d_state, domain, nsum, &T, &mode, &lds, nullable))) return s;
  if (nrows == 0) return TQ_OK;
  dim3 grid(agg_grid(nrows)), block(kAggBlock);
  // (the sums are evaluated one at a time: the kernel does not depend on their count)
  if (nullable)
    TQ_DISPATCH_AGG(mode, P.ncol, nsum, M, NC, NE, (void)NE;
                    hipLaunchKernelGGL((k_groupby<M, NC, true>), grid, block, lds, stream, P, nrows, T));
  else
    TQ_DISPATCH_AGG(mode, P.ncol, nsum, M, NC, NE, (void)NE;
                    hipLaunchKernelGGL((k_groupby<M, NC, false>), grid, block, lds, stream, P, nrows, T));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_groupby_agg(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                         const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                         hipStream_t stream) {
  return groupby_agg(d_state, domain, in, ncol, nrows, p, np, key, sums, nsum, false, stream);
}

tq_status tq_groupby_agg_nullable(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                                  const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                                  hipStream_t stream) {
  return groupby_agg(d_state, domain, in, ncol, nrows, p, np, key, sums, nsum, true, stream);
}

tq_status tq_groupby_finalize_nullable(const void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums,
                                       int64_t* d_nonnull, double* d_avg, int64_t* d_ngroups, hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (!d_keys || !d_count || !d_ngroups || !d_sums || !d_nonnull) return fail(TQ_EINVAL, "NULL output");
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, stream,
                     static_cast<StateHeader*>(const_cast<void*>(d_state)), d_keys, d_count, d_sums, d_avg, d_ngroups,
                     0, d_nonnull);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_groupby_finalize(const void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums, double* d_avg,
                              int64_t* d_ngroups, hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (!d_keys || !d_count || !d_ngroups || !d_sums) return fail(TQ_EINVAL, "NULL output");
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, stream,
                     static_cast<StateHeader*>(const_cast<void*>(d_state)), d_keys, d_count, d_sums, d_avg, d_ngroups,
                     0, nullptr);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_groupby_finalize_reset(void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums, double* d_avg,
                                    int64_t* d_ngroups, hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (!d_keys || !d_count || !d_ngroups || !d_sums) return fail(TQ_EINVAL, "NULL output");
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, stream, static_cast<StateHeader*>(d_state), d_keys,
                     d_count, d_sums, d_avg, d_ngroups, 1, nullptr);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_check(const void* d_obj, hipStream_t stream) {
  if (!d_obj) return fail(TQ_EINVAL, "object is NULL");
  TQ_HIP(hipStreamSynchronize(stream));
  uint32_t hdr[2];
  TQ_HIP(hipMemcpy(hdr, d_obj, sizeof hdr, hipMemcpyDeviceToHost));
  if (hdr[0] != kTableMagic && hdr[0] != kStateMagic && hdr[0] != kScanMagic)
    return fail(TQ_EINVAL, "not a join table, group-by state or Parquet work buffer");
  int32_t err = (int32_t)hdr[1];
  if (err) return fail(err, "%s latched by a kernel", tq_strerror(err));
  return TQ_OK;
}

size_t tq_read_peak_scratch_bytes(void) { return (size_t)8 * 4096; }

tq_status tq_read_peak(const void* d_src, size_t bytes, int64_t* d_partial, hipStream_t stream) {
  if (!d_src || !d_partial || bytes % 16) return fail(TQ_EINVAL, "bad arguments");
  int grid = std::min(device_cu_count() * 8, 4096);
  hipLaunchKernelGGL(k_read_peak, dim3(grid), dim3(kBlock), 0, stream, static_cast<const v2i64*>(d_src),
                     (int64_t)(bytes / 16), d_partial);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_fill(void* d_dst, size_t bytes, uint32_t pattern, hipStream_t stream) {
  if (!d_dst || bytes % 16) return fail(TQ_EINVAL, "bad arguments");
  hipLaunchKernelGGL(k_fill, dim3(device_cu_count() * 8), dim3(kBlock), 0, stream, static_cast<v4i32*>(d_dst),
                     (int64_t)(bytes / 16), pattern);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
