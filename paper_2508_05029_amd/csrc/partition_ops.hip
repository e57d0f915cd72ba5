// Hash partitioning: per-tile histogram -> exclusive scan over (partition, tile)
// -> per-tile scatter staged through LDS, so that each partition's run of a
// tile leaves the workgroup as one contiguous, coalesced write.
#include <mutex>

#include "common.h"

namespace tq {

constexpr int kPBlock = 256;
constexpr int kTile = 4096;            // rows per tile (one workgroup)
constexpr int kPerThread = kTile / kPBlock;
constexpr int kMaxFanoutBits = 10;
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 8;            // elements per thread in the scan kernels
constexpr int kScanChunk = kScanBlock * kScanPer;

struct PayCols {
  const void* in[TQ_MAX_COLS];
  void* out[TQ_MAX_COLS];
  int32_t w[TQ_MAX_COLS];
  int32_t n;
};

__device__ __forceinline__ uint32_t part_of(int64_t key, int skip, int bits) {
  if (bits == 0) return 0;
  return (uint32_t)((mulhash(key) << skip) >> (64 - bits));
}

__global__ __launch_bounds__(kPBlock) void k_part_hist(const int64_t* keys, int64_t n, int bits, int skip,
                                                       int64_t ntiles, int64_t* counts) {
  __shared__ uint32_t hist[1 << kMaxFanoutBits];
  const int nb = 1 << bits;
  for (int b = threadIdx.x; b < nb; b += kPBlock) hist[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int it = 0; it < kPerThread; it++) {
    int64_t r = base + (int64_t)it * kPBlock + threadIdx.x;
    if (r < n) atomicAdd(&hist[part_of(ntload(keys + r), skip, bits)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kPBlock) counts[(int64_t)b * ntiles + blockIdx.x] = hist[b];
}


__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int64_t* a, int64_t L, int64_t* bsum) {
  __shared__ int64_t ws[kScanBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int64_t t = 0;
  for (int j = 0; j < kScanPer; j++) {
    int64_t i = base + (int64_t)j * kScanBlock + threadIdx.x;
    if (i < L) t += a[i];
  }
  int64_t excl;
  int64_t total = block_excl_scan(t, &excl, ws);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(int64_t* bsum, int64_t nblk) {
  __shared__ int64_t ws[kScanBlock / kWave];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nblk; b0 += kScanBlock) {
    int64_t i = b0 + threadIdx.x;
    int64_t x = i < nblk ? bsum[i] : 0;
    int64_t excl;
    int64_t total = block_excl_scan(x, &excl, ws);
    if (i < nblk) bsum[i] = carry + excl;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(int64_t* a, int64_t L, const int64_t* bsum) {
  __shared__ int64_t ws[kScanBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer], t = 0;
  for (int j = 0; j < kScanPer; j++) {
    v[j] = base + j < L ? a[base + j] : 0;
    t += v[j];
  }
  int64_t excl;
  block_excl_scan(t, &excl, ws);
  int64_t run = bsum[blockIdx.x] + excl;
  for (int j = 0; j < kScanPer; j++) {
    if (base + j < L) a[base + j] = run;
    run += v[j];
  }
}

__global__ void k_part_offsets(const int64_t* scanned, int64_t ntiles, int nb, int64_t n, int64_t* offsets) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x)
    offsets[b] = b == nb ? n : (ntiles > 0 ? scanned[(int64_t)b * ntiles] : 0);
}

__device__ __forceinline__ int64_t load_w(const void* p, int w, int64_t r) {
  if (w == 8) return ntload(static_cast<const int64_t*>(p) + r);
  if (w == 4) return ntload(static_cast<const int32_t*>(p) + r);
  return ntload(static_cast<const uint8_t*>(p) + r);
}

__device__ __forceinline__ void store_w(void* p, int w, int64_t r, int64_t v) {
  if (w == 8) static_cast<int64_t*>(p)[r] = v;
  else if (w == 4) static_cast<int32_t*>(p)[r] = (int32_t)v;
  else static_cast<uint8_t*>(p)[r] = (uint8_t)v;
}

__global__ __launch_bounds__(kPBlock) void k_part_scatter(const int64_t* keys, int64_t n, int bits, int skip,
                                                          int64_t ntiles, const int64_t* scanned, int64_t* out_keys,
                                                          PayCols pay) {
  __shared__ int64_t buf[kTile];
  __shared__ uint16_t spid[kTile];
  __shared__ uint32_t cursor[1 << kMaxFanoutBits];
  __shared__ uint32_t start[1 << kMaxFanoutBits];
  __shared__ int64_t ws[kPBlock / kWave];
  const int nb = 1 << bits;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int rows = (int)(n - base < kTile ? n - base : kTile);
  for (int b = threadIdx.x; b < nb; b += kPBlock) cursor[b] = 0;
  __syncthreads();

  int64_t key[kPerThread];
  uint32_t pid[kPerThread], rank[kPerThread];
  for (int it = 0; it < kPerThread; it++) {
    int j = it * kPBlock + threadIdx.x;
    if (j < rows) {
      key[it] = ntload(keys + base + j);
      pid[it] = part_of(key[it], skip, bits);
      rank[it] = atomicAdd(&cursor[pid[it]], 1u);
    }
  }
  __syncthreads();
  // exclusive scan of the per-partition counts of this tile
  const int per = (nb + kPBlock - 1) / kPBlock;
  int64_t mine = 0;
  for (int q = 0; q < per; q++) {
    int b = threadIdx.x * per + q;
    if (b < nb) mine += cursor[b];
  }
  int64_t excl;
  block_excl_scan(mine, &excl, ws);
  for (int q = 0; q < per; q++) {
    int b = threadIdx.x * per + q;
    if (b < nb) {
      start[b] = (uint32_t)excl;
      excl += cursor[b];
    }
  }
  __syncthreads();
  int dest[kPerThread];
  for (int it = 0; it < kPerThread; it++) {
    int j = it * kPBlock + threadIdx.x;
    if (j < rows) {
      dest[it] = (int)(start[pid[it]] + rank[it]);
      buf[dest[it]] = key[it];
      spid[dest[it]] = (uint16_t)pid[it];
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < rows; j += kPBlock) {
    uint32_t b = spid[j];
    out_keys[scanned[(int64_t)b * ntiles + blockIdx.x] + (j - start[b])] = buf[j];
  }
  for (int c = 0; c < pay.n; c++) {
    __syncthreads();
    for (int it = 0; it < kPerThread; it++) {
      int j = it * kPBlock + threadIdx.x;
      if (j < rows) buf[dest[it]] = load_w(pay.in[c], pay.w[c], base + j);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < rows; j += kPBlock) {
      uint32_t b = spid[j];
      store_w(pay.out[c], pay.w[c], scanned[(int64_t)b * ntiles + blockIdx.x] + (j - start[b]), buf[j]);
    }
  }
}

struct PartScratch {
  int64_t ntiles, L, nblk;
  size_t bytes;
};

static PartScratch part_scratch(int64_t n, int bits) {
  PartScratch s;
  s.ntiles = (n + kTile - 1) / kTile;
  s.L = s.ntiles << bits;
  s.nblk = (s.L + kScanChunk - 1) / kScanChunk;
  s.bytes = (size_t)(s.L + s.nblk + 32) * 8;
  return s;
}

}  // namespace tq

using namespace tq;

extern "C" {

size_t tq_hash_partition_scratch_bytes(int64_t n, int32_t log2_fanout) {
  if (n < 0 || log2_fanout < 0 || log2_fanout > kMaxFanoutBits) return 0;
  return part_scratch(n, log2_fanout).bytes;
}

}  // extern "C"

namespace tq {

// The scratch of tq_hash_partition_noalloc: a fixed device array, one copy per
// GPU, held until the process ends. Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's name
// on the host is a stand-in, not a device address).
constexpr size_t kStaticScratchBytes = (size_t)TQ_PARTITION_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) int64_t scratch[kStaticScratchBytes / 8];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on each device.
static tq_status static_scratch(void** out) {
  int dev = -1;
  TQ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TQ_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(TQ_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TQ_OK;
}

static tq_status partition(const int64_t* d_keys, const tq_col* payload, int32_t npay, int64_t n, int32_t log2_fanout,
                           int32_t skip, int64_t* d_out_keys, void* const* d_out_payload, int64_t* d_offsets,
                           void* d_scratch, size_t scratch_bytes, bool static_scratch_area, hipStream_t stream) {
  if (n < 0) return fail(TQ_EINVAL, "n < 0");
  if (log2_fanout < 0 || log2_fanout > kMaxFanoutBits)
    return fail(TQ_EINVAL, "log2_fanout %d outside [0, %d]", log2_fanout, kMaxFanoutBits);
  if (skip < 0 || skip + log2_fanout > 64) return fail(TQ_EINVAL, "skip %d with %d partition bits", skip, log2_fanout);
  if (npay < 0 || npay > TQ_MAX_COLS) return fail(TQ_EINVAL, "npay %d outside [0, %d]", npay, TQ_MAX_COLS);
  if (!d_offsets) return fail(TQ_EINVAL, "offsets are NULL");
  if (n > 0 && (!d_keys || !d_out_keys)) return fail(TQ_EINVAL, "NULL keys");
  PartScratch ps = part_scratch(n, log2_fanout);
  if (static_scratch_area) {
    if (ps.bytes > kStaticScratchBytes)
      return fail(TQ_EINVAL, "%lld rows at %d partition bits need %zu bytes of scratch; the fixed area holds %zu",
                  (long long)n, log2_fanout, ps.bytes, kStaticScratchBytes);
  } else if (scratch_bytes < ps.bytes || (n > 0 && !d_scratch)) {
    return fail(TQ_EINVAL, "scratch has %zu bytes, needs %zu", scratch_bytes, ps.bytes);
  }
  PayCols pc{};
  pc.n = npay;
  for (int c = 0; c < npay; c++) {
    if (payload[c].type != TQ_U8 && payload[c].type != TQ_I32 && payload[c].type != TQ_I64)
      return fail(TQ_EINVAL, "payload %d: bad type", c);
    if (n > 0 && (!payload[c].data || !d_out_payload || !d_out_payload[c])) return fail(TQ_EINVAL, "payload %d: NULL", c);
    pc.in[c] = payload[c].data;
    pc.out[c] = d_out_payload[c];
    pc.w[c] = payload[c].type;
  }
  if (static_scratch_area) {  // arguments are valid: only now look the area up
    tq_status s = static_scratch(&d_scratch);
    if (s) return s;
  }
  const int nb = 1 << log2_fanout;
  // every word of the scratch that a kernel reads was written by an earlier kernel of
  // this call (the histogram fills all (partition, tile) counts), so nothing is cleared
  int64_t* counts = static_cast<int64_t*>(d_scratch);
  int64_t* bsum = counts + ps.L;
  if (n > 0) {
    hipLaunchKernelGGL(k_part_hist, dim3((unsigned)ps.ntiles), dim3(kPBlock), 0, stream, d_keys, n, log2_fanout, skip,
                       ps.ntiles, counts);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ps.nblk), dim3(kScanBlock), 0, stream, counts, ps.L, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, stream, bsum, ps.nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ps.nblk), dim3(kScanBlock), 0, stream, counts, ps.L, bsum);
    hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)ps.ntiles), dim3(kPBlock), 0, stream, d_keys, n, log2_fanout, skip,
                       ps.ntiles, counts, d_out_keys, pc);
  }
  hipLaunchKernelGGL(k_part_offsets, dim3((nb + 1 + 255) / 256), dim3(256), 0, stream, counts, ps.ntiles, nb, n,
                     d_offsets);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // namespace tq

extern "C" {

tq_status tq_hash_partition(const int64_t* d_keys, const tq_col* payload, int32_t npay, int64_t n, int32_t log2_fanout,
                            int32_t skip, int64_t* d_out_keys, void* const* d_out_payload, int64_t* d_offsets,
                            void* d_scratch, size_t scratch_bytes, hipStream_t stream) {
  return partition(d_keys, payload, npay, n, log2_fanout, skip, d_out_keys, d_out_payload, d_offsets, d_scratch,
                   scratch_bytes, false, stream);
}

tq_status tq_hash_partition_noalloc(const int64_t* d_keys, const tq_col* payload, int32_t npay, int64_t n,
                                    int32_t log2_fanout, int32_t skip, int64_t* d_out_keys,
                                    void* const* d_out_payload, int64_t* d_offsets, hipStream_t stream) {
  return partition(d_keys, payload, npay, n, log2_fanout, skip, d_out_keys, d_out_payload, d_offsets, nullptr, 0, true,
                   stream);
}

}  // extern "C"
