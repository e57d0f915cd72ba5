// Dictionary-encoded string keys: joins between string columns encoded
// against different dictionaries, by mapping one dictionary onto the other.
//
// A dictionary's entries are distinct strings, so the build dictionary goes
// into an ordinary join table keyed by a 64-bit hash of each string's bytes
// (two distinct strings with one hash are two rows of one key, as with any
// duplicate build key). Every probe dictionary entry walks the entries of its
// hash and compares bytes with each, so the mapping is exact whatever the
// hash collisions. The join itself then runs on integer codes.
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
