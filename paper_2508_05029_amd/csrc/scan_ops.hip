// Filter / project, group-by accumulation and finalization, and the two
// measurement kernels (streaming read, cache-evicting fill).
#include <string.h>

#include "common.h"
#include "groupby.h"

namespace tq {

constexpr int kBlock = 256;

static int stream_blocks(int64_t n, int per_cu) {
  int64_t want = (n + (int64_t)kBlock * kRows - 1) / ((int64_t)kBlock * kRows);
  int64_t cap = (int64_t)device_cu_count() * per_cu;
  if (want < 1) want = 1;
  return (int)(want < cap ? want : cap);
}

__global__ void k_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------ filter/project

struct OutPtrs {
  int64_t* p[TQ_MAX_SUMS];
};

__global__ __launch_bounds__(kBlock) void k_filter_project(RowPlan P, int64_t n, OutPtrs out, int64_t* sel,
                                                           unsigned long long* count) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 - (int64_t)threadIdx.x * kRows < n;
       r0 += step) {
    // every lane of the wave takes part in the scan, also past the end
    bool full = r0 + kRows <= n;
    int64_t v[TQ_MAX_COLS][kRows];
#pragma unroll
    for (int c = 0; c < TQ_MAX_COLS; c++)
      if (c < P.ncol && r0 < n) load4(P.col[c], r0, full, n, v[c]);
    bool ok[kRows];
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      ok[i] = (r0 + i < n) && eval_preds(P, vals);
      mine += ok[i];
    }
    uint32_t total;
    uint32_t pre = wave_excl_scan(mine, &total);
    unsigned long long base = 0;
    if (__lane_id() == kWave - 1 && total) base = atomicAdd(count, (unsigned long long)total);
    base = __shfl(base, kWave - 1, kWave);
    int64_t w = (int64_t)base + pre;
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      if (!ok[i]) continue;
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      for (int e = 0; e < P.ne; e++) out.p[e][w] = eval_expr(P.expr[e], vals);
      if (sel) sel[w] = r0 + i;
      w++;
    }
  }
}

// ------------------------------------------------------------ group-by

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_groupby(RowPlan P, int64_t n, AggTarget T) {
  extern __shared__ __align__(16) char smem[];
  if (!state_matches(T)) return;
  LdsAgg<MODE> agg;
  agg.init(T, smem);
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    bool full = r0 + kRows <= n;
    int64_t v[TQ_MAX_COLS][kRows];
#pragma unroll
    for (int c = 0; c < TQ_MAX_COLS; c++)
      if (c < P.ncol) load4(P.col[c], r0, full, n, v[c]);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      if (r0 + i >= n) break;
      int64_t vals[TQ_MAX_COLS];
#pragma unroll
      for (int c = 0; c < TQ_MAX_COLS; c++) vals[c] = v[c][i];
      if (!eval_preds(P, vals)) continue;
      int64_t s[TQ_MAX_SUMS];
#pragma unroll
      for (int e = 0; e < TQ_MAX_SUMS; e++)
        if (e < P.ne) s[e] = eval_expr(P.expr[e], vals);
      agg.add(T, eval_key(P, vals), s, P.ne);
    }
  }
  agg.flush(T);
}

__global__ void k_state_init(StateHeader* h, int64_t domain, int32_t nsum, int32_t replicas, int64_t entries) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->magic = kStateMagic;
    h->err = 0;
    h->domain = domain;
    h->nsum = nsum;
    h->replicas = replicas;
    h->matches = 0;
  }
  int64_t* d = state_data(h);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = 0;
}

// One workgroup: sum the replicas, keep COUNT > 0, emit in key order.
constexpr int kFinBlock = 1024;

__global__ __launch_bounds__(kFinBlock) void k_finalize(const StateHeader* h, int64_t* keys, int64_t* count,
                                                        int64_t* sums, double* avg, int64_t* ngroups) {
  __shared__ uint32_t wave_tot[kFinBlock / kWave];
  __shared__ int64_t base_s;
  const int64_t domain = h->domain;
  const int nsum = h->nsum, stride = 1 + nsum, R = h->replicas;
  const int64_t rstride = domain * stride;
  const int64_t* d = state_data(const_cast<StateHeader*>(h));
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  const int wid = threadIdx.x / kWave, lane = __lane_id();
  for (int64_t k0 = 0; k0 < domain; k0 += kFinBlock) {
    int64_t k = k0 + threadIdx.x;
    int64_t e[1 + TQ_MAX_SUMS];
    bool live = false;
    if (k < domain) {
      for (int j = 0; j < stride; j++) {
        uint64_t acc = 0;
        for (int r = 0; r < R; r++) acc += (uint64_t)d[r * rstride + k * stride + j];
        e[j] = (int64_t)acc;
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
      for (int j = 0; j < nsum; j++) {
        sums[g * nsum + j] = e[1 + j];
        if (avg) avg[g * nsum + j] = (double)e[1 + j] / (double)e[0];
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
  if (threadIdx.x == 0) *ngroups = base_s;
}

// ------------------------------------------------------------ measurement

__global__ __launch_bounds__(kBlock) void k_read_peak(const v2i64* src, int64_t n16, unsigned long long* sink) {
  long long acc = 0;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * step < n16; i += 4 * step) {
    v2i64 a = ntload(src + i), b = ntload(src + i + step), c = ntload(src + i + 2 * step), e = ntload(src + i + 3 * step);
    acc ^= a.x + a.y + b.x + b.y + c.x + c.y + e.x + e.y;
  }
  for (; i < n16; i += step) {
    v2i64 a = ntload(src + i);
    acc ^= a.x + a.y;
  }
  for (int d = 32; d > 0; d >>= 1) acc ^= __shfl_xor(acc, d, kWave);
  if (__lane_id() == 0) atomicAdd(sink, (unsigned long long)acc);
}

__global__ __launch_bounds__(kBlock) void k_fill(v4i32* dst, int64_t n16, uint32_t pattern) {
  v4i32 v = {(int)pattern, (int)pattern, (int)pattern, (int)pattern};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(v, dst + i);
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_filter_project(const tq_col* in, int32_t ncol, int64_t nrows, const tq_pred* p, int32_t np,
                            const tq_expr* e, int32_t ne, int64_t* const* d_out, int64_t* d_sel, int64_t* d_out_rows,
                            hipStream_t stream) {
  RowPlan P;
  tq_status s = make_plan(&P, in, ncol, p, np, e, ne, nullptr, nrows);
  if (s) return s;
  if (!d_out_rows) return fail(TQ_EINVAL, "d_out_rows is NULL");
  OutPtrs out{};
  for (int j = 0; j < ne; j++) {
    if (!d_out || !d_out[j]) return fail(TQ_EINVAL, "output %d is NULL", j);
    out.p[j] = d_out[j];
  }
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, stream, d_out_rows, (int64_t)1);
  TQ_HIP(hipGetLastError());
  if (nrows == 0) return TQ_OK;
  hipLaunchKernelGGL(k_filter_project, dim3(stream_blocks(nrows, 8)), dim3(kBlock), 0, stream, P, nrows, out, d_sel,
                     reinterpret_cast<unsigned long long*>(d_out_rows));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

size_t tq_groupby_state_bytes(int64_t domain, int32_t nsum) {
  if (domain <= 0 || nsum < 0 || nsum > TQ_MAX_SUMS) return 0;
  int stride = 1 + nsum;
  return kHeaderBytes + (size_t)choose_replicas(domain, stride) * (size_t)domain * stride * 8;
}

tq_status tq_groupby_init(void* d_state, size_t bytes, int64_t domain, int32_t nsum, hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "state is NULL");
  if (domain <= 0 || domain > (int64_t)1 << 31) return fail(TQ_EINVAL, "domain %lld outside [1, 2^31]", (long long)domain);
  if (nsum < 0 || nsum > TQ_MAX_SUMS) return fail(TQ_EINVAL, "nsum %d outside [0, %d]", nsum, TQ_MAX_SUMS);
  size_t need = tq_groupby_state_bytes(domain, nsum);
  if (bytes < need) return fail(TQ_EINVAL, "state buffer has %zu bytes, needs %zu", bytes, need);
  int stride = 1 + nsum;
  int R = choose_replicas(domain, stride);
  int64_t entries = (int64_t)R * domain * stride;
  int blocks = (int)std::min<int64_t>((entries + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_state_init, dim3(blocks), dim3(kBlock), 0, stream, static_cast<StateHeader*>(d_state), domain,
                     nsum, R, entries);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"

namespace tq {

tq_status make_target(void* d_state, int64_t domain, int32_t nsum, AggTarget* T, AggMode* mode, size_t* lds) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (domain <= 0 || domain > ((int64_t)1 << 31)) return fail(TQ_EINVAL, "domain %lld outside [1, 2^31]", (long long)domain);
  if (nsum < 0 || nsum > TQ_MAX_SUMS) return fail(TQ_EINVAL, "nsum %d outside [0, %d]", nsum, TQ_MAX_SUMS);
  T->hdr = static_cast<const StateHeader*>(d_state);
  T->data = state_data(d_state);
  T->err = &static_cast<StateHeader*>(d_state)->err;
  T->domain = domain;
  T->stride = 1 + nsum;
  T->replicas = choose_replicas(domain, 1 + nsum);
  *mode = agg_mode(domain, 1 + nsum, &T->log2hcap, lds);
  return TQ_OK;
}

}  // namespace tq

extern "C" {

tq_status tq_groupby_agg(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                         const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                         hipStream_t stream) {
  if (!key) return fail(TQ_EINVAL, "group key is NULL");
  RowPlan P;
  tq_status s = make_plan(&P, in, ncol, p, np, sums, nsum, key, nrows);
  if (s) return s;
  AggTarget T;
  AggMode mode;
  size_t lds;
  if ((s = make_target(d_state, domain, nsum, &T, &mode, &lds))) return s;
  if (nrows == 0) return TQ_OK;
  dim3 grid(stream_blocks(nrows, 4)), block(kBlock);
  if (mode == kDense) hipLaunchKernelGGL(k_groupby<kDense>, grid, block, lds, stream, P, nrows, T);
  else if (mode == kHash) hipLaunchKernelGGL(k_groupby<kHash>, grid, block, lds, stream, P, nrows, T);
  else hipLaunchKernelGGL(k_groupby<kGlobal>, grid, block, 0, stream, P, nrows, T);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_groupby_finalize(const void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums, double* d_avg,
                              int64_t* d_ngroups, hipStream_t stream) {
  if (!d_state) return fail(TQ_EINVAL, "group-by state is NULL");
  if (!d_keys || !d_count || !d_ngroups || !d_sums) return fail(TQ_EINVAL, "NULL output");
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinBlock), 0, stream, static_cast<const StateHeader*>(d_state),
                     d_keys, d_count, d_sums, d_avg, d_ngroups);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_check(const void* d_obj, hipStream_t stream) {
  if (!d_obj) return fail(TQ_EINVAL, "object is NULL");
  TQ_HIP(hipStreamSynchronize(stream));
  uint32_t hdr[2];
  TQ_HIP(hipMemcpy(hdr, d_obj, sizeof hdr, hipMemcpyDeviceToHost));
  if (hdr[0] != kTableMagic && hdr[0] != kStateMagic) return fail(TQ_EINVAL, "not a join table or group-by state");
  int32_t err = (int32_t)hdr[1];
  if (err) return fail(err, "%s latched by a kernel", tq_strerror(err));
  return TQ_OK;
}

tq_status tq_read_peak(const void* d_src, size_t bytes, int64_t* d_sink, hipStream_t stream) {
  if (!d_src || !d_sink || bytes % 16) return fail(TQ_EINVAL, "bad arguments");
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, stream, d_sink, (int64_t)1);
  hipLaunchKernelGGL(k_read_peak, dim3(device_cu_count() * 8), dim3(kBlock), 0, stream,
                     static_cast<const v2i64*>(d_src), (int64_t)(bytes / 16), reinterpret_cast<unsigned long long*>(d_sink));
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
