// String keys. Dictionary-encoded columns: joins between string columns
// encoded against different dictionaries, by mapping one dictionary onto the
// other. Plain string columns: dictionary encoding on the GPU (equal strings
// get one code), after which group-by and joins run on the codes.
//
// A dictionary's entries are distinct strings, so the build dictionary goes
// into an ordinary join table keyed by a 64-bit hash of each string's bytes
// (two distinct strings with one hash are two rows of one key, as with any
// duplicate build key). Every probe dictionary entry walks the entries of its
// hash and compares bytes with each, so the mapping is exact whatever the
// hash collisions. The join itself then runs on integer codes.
#include <hipcub/hipcub.hpp>

#include "common.h"
#include "table.h"

namespace tq {

constexpr int kStrBlock = 256;

// FNV-1a over the string's bytes (64-bit offset basis and prime).
__device__ __forceinline__ uint64_t str_hash(const uint8_t* p, int32_t len) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (int32_t i = 0; i < len; i++) h = (h ^ p[i]) * 0x100000001b3ull;
  return h;
}

// Byte equality, kept out of line: inlined into the table walk below, hipcc
// (ROCm 7.2, -O3) emitted code that lost the matched entry's number after the
// byte loop (its register was reused for the loop's pointer), so no non-empty
// string ever matched. The call costs nothing that matters here: the walk
// runs once per dictionary entry, not per row.
__device__ __attribute__((noinline)) bool str_equal(const uint8_t* a, int32_t la, const uint8_t* b, int32_t lb) {
  if (la != lb) return false;
  uint32_t diff = 0;
  for (int32_t i = 0; i < la; i++) diff |= (uint32_t)(a[i] ^ b[i]);
  return diff == 0;
}

__global__ __launch_bounds__(kStrBlock) void k_str_keys(const int32_t* off, const uint8_t* data, int64_t n,
                                                        int64_t* keys, int64_t* pay) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = off[i], b = off[i + 1];
    keys[i] = (int64_t)str_hash(data + a, b - a);
    pay[i] = i;
  }
}

// remap[i] = the build entry whose bytes equal probe entry i, or -1.
__global__ __launch_bounds__(kStrBlock) void k_dict_probe(const TableHeader* h, const int32_t* boff,
                                                          const uint8_t* bdata, const int32_t* poff,
                                                          const uint8_t* pdata, int64_t n, int32_t* remap) {
  if (h->magic != kTableMagic || h->err) return;
  Probe pr;
  pr.setup(h);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = poff[i], len = poff[i + 1] - a;
    const uint8_t* s = pdata + a;
    bool ok[1] = {true};
    int64_t k[1] = {(int64_t)str_hash(s, len)};
    int32_t found = -1;
    pr.walk(ok, k, [&](const bool (&hit)[1], const int64_t (&pay)[1]) {
      const int64_t j = pay[0];
      bool eq = false;
      if (hit[0] && found < 0) {
        const int32_t ba = boff[j];
        eq = str_equal(bdata + ba, boff[j + 1] - ba, s, len);
      }
      found = eq ? (int32_t)j : found;
    });
    remap[i] = found;
  }
}

__global__ __launch_bounds__(kStrBlock) void k_dict_keys(const int32_t* codes, const uint8_t* valid, int64_t n,
                                                         const int32_t* remap, int64_t n_remap, int64_t* keys) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = codes[r];
    int64_t k = -1;
    if (!valid || bit_at(valid, r)) {
      if (!remap) k = c < 0 ? -1 : c;
      else if (c >= 0 && (int64_t)c < n_remap) k = remap[c];
    }
    keys[r] = k;
  }
}

static int str_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kStrBlock - 1) / kStrBlock, (int64_t)device_cu_count() * 8));
}


// ------------------------------------------------------------ dictionary encoding
//
// Rows are sorted by (hash, row) (a stable radix sort of the 64-bit hashes),
// so equal strings lie together in a run of one hash, in row order. A run
// whose strings all equal its first is one code; a run holding different
// strings (a hash collision) is split by one thread comparing bytes. Codes
// are numbered in hash order; each code's first row is its smallest.

constexpr int kMaxCollide = 16;  // distinct strings that may share one 64-bit hash
constexpr uint32_t kRepBit = 0x80000000u;

__global__ __launch_bounds__(kStrBlock) void k_enc_heads(const uint64_t* skeys, int64_t n, int32_t* head) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    head[p] = p == 0 || skeys[p] != skeys[p - 1];
}

// runid1: inclusive sum of the heads (run number + 1)
__global__ __launch_bounds__(kStrBlock) void k_enc_starts(const int32_t* head, const int32_t* runid1, int64_t n,
                                                          int32_t* start, int32_t* impure) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    if (head[p]) {
      start[runid1[p] - 1] = (int32_t)p;
      impure[runid1[p] - 1] = 0;
    }
}

__global__ __launch_bounds__(kStrBlock) void k_enc_pure(const int32_t* off, const uint8_t* data, const int32_t* svals,
                                                        const int32_t* runid1, const int32_t* start, int64_t n,
                                                        int32_t* impure) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = runid1[p] - 1, s0 = start[r];
    if (s0 == p) continue;
    const int32_t a = svals[p], b = svals[s0];
    if (!str_equal(data + off[a], off[a + 1] - off[a], data + off[b], off[b + 1] - off[b])) impure[r] = 1;
  }
}

// One thread per run: the code count of the run, and for a run of several
// strings, each position's code within the run (kRepBit on a code's first).
__global__ __launch_bounds__(kStrBlock) void k_enc_split(const int32_t* off, const uint8_t* data, const int32_t* svals,
                                                         const int32_t* start, const int32_t* impure,
                                                         const int32_t* nruns_p, int64_t n, uint32_t* sub,
                                                         int32_t* nsub, int32_t* err) {
  const int32_t nruns = *nruns_p;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += gridDim.x * blockDim.x) {
    if (!impure[r]) {
      nsub[r] = 1;
      continue;
    }
    const int32_t p0 = start[r], p1 = r + 1 < nruns ? start[r + 1] : (int32_t)n;
    int32_t rep[kMaxCollide], k = 0;
    for (int32_t p = p0; p < p1; p++) {
      const int32_t a = svals[p];
      int32_t j = 0;
      for (; j < k; j++) {
        const int32_t b = svals[rep[j]];
        if (str_equal(data + off[a], off[a + 1] - off[a], data + off[b], off[b + 1] - off[b])) break;
      }
      if (j == k) {
        if (k == kMaxCollide) {
          atomicCAS(err, 0, TQ_EINVAL);
          break;
        }
        rep[k++] = p;
        sub[p] = (uint32_t)j | kRepBit;
      } else {
        sub[p] = (uint32_t)j;
      }
    }
    nsub[r] = k;
  }
}

// base: exclusive sum of nsub over the runs
__global__ __launch_bounds__(kStrBlock) void k_enc_codes(const int32_t* svals, const int32_t* runid1,
                                                         const int32_t* start, const int32_t* impure,
                                                         const uint32_t* sub, const int32_t* base, int64_t n,
                                                         int32_t* codes, int32_t* first_rows) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = runid1[p] - 1;
    const bool imp = impure[r] != 0;
    const uint32_t sb = imp ? sub[p] : 0u;
    const int32_t c = base[r] + (int32_t)(sb & ~kRepBit);
    codes[svals[p]] = c;
    if (imp ? (sb & kRepBit) != 0 : start[r] == p) first_rows[c] = svals[p];
  }
}

__global__ void k_enc_total(const int32_t* runid1, const int32_t* nsub, const int32_t* base, int64_t n, int64_t* ndict,
                            const int32_t* err) {
  if (n == 0) *ndict = 0;
  else {
    const int32_t last = runid1[n - 1] - 1;
    *ndict = *err ? -1 : (int64_t)base[last] + nsub[last];
  }
}

// Scratch of an encoding of n strings: the sort's and the scans' temporary
// storage, then the arrays.
struct EncLayout {
  size_t sort_tmp, scan_tmp, keys, skeys, vals, svals, head, runid1, start, impure, sub, nsub, base, err, total;
};

static EncLayout enc_layout(int64_t n) {
  EncLayout L{};
  size_t sort_tmp = 0, scan_tmp = 0, scan2 = 0;
  const int ni = (int)std::max<int64_t>(n, 1);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_tmp, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, ni);
  (void)hipcub::DeviceScan::InclusiveSum(nullptr, scan_tmp, (const int32_t*)nullptr, (int32_t*)nullptr, ni);
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan2, (const int32_t*)nullptr, (int32_t*)nullptr, ni);
  auto a = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  size_t at = 0;
  L.sort_tmp = at;
  at += a(sort_tmp);
  L.scan_tmp = at;
  at += a(std::max(scan_tmp, scan2));
  L.keys = at;
  at += a(nn * 8);
  L.skeys = at;
  at += a(nn * 8);
  L.vals = at;
  at += a(nn * 4);
  L.svals = at;
  at += a(nn * 4);
  L.head = at;
  at += a(nn * 4);
  L.runid1 = at;
  at += a(nn * 4);
  L.start = at;
  at += a(nn * 4);
  L.impure = at;
  at += a(nn * 4);
  L.sub = at;
  at += a(nn * 4);
  L.nsub = at;
  at += a(nn * 4);
  L.base = at;
  at += a(nn * 4);
  L.err = at;
  at += 256;
  L.total = at + 256;  // the caller's pointer is aligned up to 256 inside
  (void)scan2;
  return L;
}

__global__ __launch_bounds__(kStrBlock) void k_enc_hash(const int32_t* off, const uint8_t* data, int64_t n,
                                                        uint64_t* keys, int32_t* vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = str_hash(data + off[i], off[i + 1] - off[i]);
    vals[i] = (int32_t)i;
  }
}

__global__ void k_enc_zero(int32_t* p) { *p = 0; }

// nsub of the positions past the last run: 0, so that the scan over n entries is defined
__global__ __launch_bounds__(kStrBlock) void k_enc_fill(int32_t* nsub, const int32_t* nruns_p, int64_t n) {
  const int32_t nruns = *nruns_p;
  for (int64_t r = nruns + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    nsub[r] = 0;
}
}  // namespace tq

using namespace tq;

extern "C" {

size_t tq_dict_unify_scratch_bytes(int64_t n_build) {
  if (n_build < 0) return 0;
  return (size_t)(n_build + 2) * 16 + 256;
}

tq_status tq_dict_unify(void* d_table, size_t table_bytes, tq_strings build, tq_strings probe, void* d_scratch,
                        size_t scratch_bytes, int32_t* d_remap, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (build.n < 0 || probe.n < 0) return fail(TQ_EINVAL, "negative string count");
  if (build.n > INT32_MAX - 1) return fail(TQ_EINVAL, "build dictionary of %lld entries (int32 codes)", (long long)build.n);
  if ((build.n > 0 && (!build.offsets || !build.data)) || (probe.n > 0 && (!probe.offsets || !probe.data)))
    return fail(TQ_EINVAL, "NULL string column");
  if (probe.n > 0 && !d_remap) return fail(TQ_EINVAL, "d_remap is NULL");
  if (!d_scratch || scratch_bytes < tq_dict_unify_scratch_bytes(build.n))
    return fail(TQ_EINVAL, "scratch needs %zu bytes", tq_dict_unify_scratch_bytes(build.n));
  // the hashes and entry numbers of the build dictionary, 16-byte aligned
  char* sc = reinterpret_cast<char*>(((uintptr_t)d_scratch + 15) & ~(uintptr_t)15);
  int64_t* keys = reinterpret_cast<int64_t*>(sc);
  int64_t* pay = keys + ((build.n + 1) & ~(int64_t)1);
  if (build.n > 0) {
    hipLaunchKernelGGL(k_str_keys, dim3(str_grid(build.n)), dim3(kStrBlock), 0, stream, build.offsets, build.data,
                       build.n, keys, pay);
    TQ_HIP(hipGetLastError());
  }
  tq_status s;
  if ((s = tq_join_table_init(d_table, table_bytes, stream))) return s;
  // a hash shared by distinct strings makes duplicate keys: the table keeps every row
  if ((s = tq_join_build(d_table, table_bytes, keys, tq_col{pay, TQ_I64, nullptr}, build.n, nullptr, 0, nullptr, 0, 0.5,
                         0, 0u, stream)))
    return s;
  if (probe.n > 0) {
    hipLaunchKernelGGL(k_dict_probe, dim3(str_grid(probe.n)), dim3(kStrBlock), 0, stream,
                       static_cast<const TableHeader*>(d_table), build.offsets, build.data, probe.offsets, probe.data,
                       probe.n, d_remap);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

size_t tq_dict_encode_scratch_bytes(int64_t n) {
  if (n < 0 || n > INT32_MAX - 1) return 0;
  return enc_layout(n).total;
}

tq_status tq_dict_encode(tq_strings in, void* d_scratch, size_t scratch_bytes, int32_t* d_codes, int32_t* d_first_rows,
                         int64_t* d_ndict, hipStream_t stream) {
  if (in.n < 0 || in.n > INT32_MAX - 1) return fail(TQ_EINVAL, "string count %lld", (long long)in.n);
  if (in.n > 0 && (!in.offsets || !in.data || !d_codes || !d_first_rows)) return fail(TQ_EINVAL, "NULL column or output");
  if (!d_ndict) return fail(TQ_EINVAL, "d_ndict is NULL");
  const EncLayout L = enc_layout(in.n);
  if (!d_scratch || scratch_bytes < L.total) return fail(TQ_EINVAL, "scratch needs %zu bytes", L.total);
  char* S = reinterpret_cast<char*>(((uintptr_t)d_scratch + 255) & ~(uintptr_t)255);
  const int64_t n = in.n;
  auto* keys = reinterpret_cast<uint64_t*>(S + L.keys);
  auto* skeys = reinterpret_cast<uint64_t*>(S + L.skeys);
  auto* vals = reinterpret_cast<int32_t*>(S + L.vals);
  auto* svals = reinterpret_cast<int32_t*>(S + L.svals);
  auto* head = reinterpret_cast<int32_t*>(S + L.head);
  auto* runid1 = reinterpret_cast<int32_t*>(S + L.runid1);
  auto* start = reinterpret_cast<int32_t*>(S + L.start);
  auto* impure = reinterpret_cast<int32_t*>(S + L.impure);
  auto* sub = reinterpret_cast<uint32_t*>(S + L.sub);
  auto* nsub = reinterpret_cast<int32_t*>(S + L.nsub);
  auto* base = reinterpret_cast<int32_t*>(S + L.base);
  auto* err = reinterpret_cast<int32_t*>(S + L.err);
  hipLaunchKernelGGL(k_enc_zero, dim3(1), dim3(1), 0, stream, err);
  if (n > 0) {
    const dim3 g(str_grid(n)), b(kStrBlock);
    hipLaunchKernelGGL(k_enc_hash, g, b, 0, stream, in.offsets, in.data, n, keys, vals);
    size_t tb = L.scan_tmp - L.sort_tmp;
    TQ_HIP(hipcub::DeviceRadixSort::SortPairs(S + L.sort_tmp, tb, keys, skeys, vals, svals, (int)n, 0, 64, stream));
    hipLaunchKernelGGL(k_enc_heads, g, b, 0, stream, skeys, n, head);
    size_t sb = L.keys - L.scan_tmp;
    TQ_HIP(hipcub::DeviceScan::InclusiveSum(S + L.scan_tmp, sb, head, runid1, (int)n, stream));
    hipLaunchKernelGGL(k_enc_starts, g, b, 0, stream, head, runid1, n, start, impure);
    hipLaunchKernelGGL(k_enc_pure, g, b, 0, stream, in.offsets, in.data, svals, runid1, start, n, impure);
    // the run count is runid1[n - 1]; the run kernels read it on the device
    hipLaunchKernelGGL(k_enc_split, g, b, 0, stream, in.offsets, in.data, svals, start, impure, runid1 + (n - 1), n, sub,
                       nsub, err);
    // runs past the last hold no codes: the scan over n entries reads only what the split wrote below nruns
    hipLaunchKernelGGL(k_enc_fill, g, b, 0, stream, nsub, runid1 + (n - 1), n);
    sb = L.keys - L.scan_tmp;
    TQ_HIP(hipcub::DeviceScan::ExclusiveSum(S + L.scan_tmp, sb, nsub, base, (int)n, stream));
    hipLaunchKernelGGL(k_enc_codes, g, b, 0, stream, svals, runid1, start, impure, sub, base, n, d_codes, d_first_rows);
  }
  hipLaunchKernelGGL(k_enc_total, dim3(1), dim3(1), 0, stream, runid1, nsub, base, n, d_ndict, err);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_dict_keys(const int32_t* d_codes, const uint8_t* d_valid, int64_t n, const int32_t* d_remap,
                       int64_t n_remap, int64_t* d_keys, hipStream_t stream) {
  if (n < 0 || n_remap < 0) return fail(TQ_EINVAL, "negative count");
  if (n > 0 && (!d_codes || !d_keys)) return fail(TQ_EINVAL, "NULL codes or keys");
  if (n_remap > 0 && !d_remap) return fail(TQ_EINVAL, "NULL remap");
  if (n == 0) return TQ_OK;
  hipLaunchKernelGGL(k_dict_keys, dim3(str_grid(n)), dim3(kStrBlock), 0, stream, d_codes, d_valid, n,
                     n_remap > 0 ? d_remap : nullptr, n_remap, d_keys);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
