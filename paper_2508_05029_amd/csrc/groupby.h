// Group-by partials: per-workgroup in LDS, then folded into the global state.
//
// LDS modes (chosen on the host from the key domain and the entry width):
//   kDense   the whole domain fits in LDS: direct-indexed int64 partials
//   kHash    an LDS open-addressing table of hot keys (Zipf-skewed groups stay
//            on chip); a row whose key finds no LDS slot within a few probes
//            goes straight to a global atomic
// Global layouts of the state data (entry e = key * stride + j, value 0 is
// COUNT, values 1..nsum the SUMs):
//   rows = kAggRows  small domains: one private row per workgroup slot,
//                    data[b * entries + e]; workgroup b adds its LDS partials
//                    to row b with plain loads and stores (calls on one state
//                    are stream ordered, so rows are never written
//                    concurrently) and finalization folds the rows
//   rows = 1         large domains: one shared table updated with atomics,
//                    whose addresses are spread over the whole domain
#pragma once

#include <type_traits>

#include "common.h"

namespace tq {

enum AggMode { kDense = 0, kHash = 1 };

constexpr int kLdsAggBytes = 32 * 1024;
constexpr int kHashProbes = 8;
constexpr int kAggRows = 1024;            // grid cap of the aggregating kernels
constexpr int kPrivateRowsMaxEntries = 1024;
constexpr int kAggBlock = 512;            // threads per aggregating workgroup
constexpr int kAggBlocksPerCU = 3;
constexpr int kMaxNullableSums = TQ_MAX_SUMS / 2;  // a nullable state keeps SUM_j and COUNT_j per sum

struct AggTarget {
  const StateHeader* hdr;
  int64_t* data;
  int32_t* err;
  int64_t domain;
  int32_t stride;   // 1 + nsum (nullable: 1 + 2 * nsum)
  int32_t rows;     // kAggRows or 1
  int32_t log2hcap; // kHash: LDS slots = 1 << log2hcap
  int32_t nullable; // 1: the state of tq_groupby_init_nullable
  int64_t udomain;  // keys of the caller's domain (nullable: domain - 1, the last group being NULL)
};

inline int state_rows(int64_t domain, int stride) {
  return domain * stride <= kPrivateRowsMaxEntries ? kAggRows : 1;
}

// Host: pick the LDS mode and its dynamic LDS size.
__host__ __device__ inline AggMode agg_mode(int64_t domain, int stride, int* log2hcap, size_t* lds_bytes) {
  if (domain * stride * 8 <= kLdsAggBytes) {
    *log2hcap = 0;
    *lds_bytes = (size_t)domain * stride * 8;
    return kDense;
  }
  int per_slot = 4 + stride * 8;
  int l = 6;
  while ((size_t)(2 << l) * per_slot <= (size_t)kLdsAggBytes && l < 14) l++;
  *log2hcap = l;
  *lds_bytes = ((size_t)(1 << l) * 4 + 15) / 16 * 16 + (size_t)(1 << l) * stride * 8;
  return kHash;
}

// The launch must describe the state the buffer was initialised with;
// otherwise the kernel writes nothing and latches TQ_EINVAL.
__device__ __forceinline__ bool state_matches(const AggTarget& T) {
  const StateHeader* h = T.hdr;
  if (h->magic != kStateMagic) return false;
  if (h->domain != T.domain || h->nsum != T.stride - 1 || h->rows != T.rows || h->nullable != T.nullable) {
    if (threadIdx.x == 0 && blockIdx.x == 0) latch_error(T.err, TQ_EINVAL);
    return false;
  }
  return true;
}

__device__ __forceinline__ void global_add(unsigned long long* p, int64_t v) {
  atomicAdd(p, (unsigned long long)v);
}

template <int MODE>
struct LdsAgg {
  int64_t* vals;   // LDS. kDense: [domain][stride]; kHash: [hcap][stride]
  uint32_t* keys;  // LDS. kHash: key + 1, 0 = empty
  // Deferred mode: a key outside the domain is remembered here and latched by
  // flush(), so that the adding loop issues no device-memory atomic (on this
  // GPU a store or atomic shares the wait counter with loads, and its mere
  // presence in a loop makes every wait for a load a wait for all of them).
  bool defer = false;
  bool bad = false;

  __device__ void init(const AggTarget& T, char* smem) {
    if (MODE == kDense) {
      vals = reinterpret_cast<int64_t*>(smem);
      for (int i = threadIdx.x; i < T.domain * T.stride; i += blockDim.x) vals[i] = 0;
    } else {
      int hcap = 1 << T.log2hcap;
      keys = reinterpret_cast<uint32_t*>(smem);
      vals = reinterpret_cast<int64_t*>(smem + (((size_t)hcap * 4 + 15) / 16 * 16));
      for (int i = threadIdx.x; i < hcap; i += blockDim.x) keys[i] = 0;
      for (int i = threadIdx.x; i < hcap * T.stride; i += blockDim.x) vals[i] = 0;
    }
  }

  // COUNT += 1 and SUM_j += v[j] for group `key` (j < nsum <= NE).
  template <int NE>
  __device__ __forceinline__ void add(const AggTarget& T, int64_t key, const int64_t (&v)[NE], int nsum) {
    if ((uint64_t)key >= (uint64_t)T.domain) {
      if (defer) bad = true;
      else latch_error(T.err, TQ_EDOMAIN);
      return;
    }
    if (MODE == kDense) {
      unsigned long long* d = reinterpret_cast<unsigned long long*>(vals + key * T.stride);
      atomicAdd(d, 1ull);
#pragma unroll
      for (int j = 0; j < NE; j++)
        if (j < nsum) atomicAdd(d + 1 + j, (unsigned long long)v[j]);
    } else {
      uint32_t k1 = (uint32_t)key + 1u;
      uint32_t mask = (1u << T.log2hcap) - 1u;
      uint32_t s = ((uint32_t)key * 0x9E3779B1u) >> (32 - T.log2hcap);
      int found = -1;
      for (int i = 0; i < kHashProbes; i++) {
        uint32_t cur = keys[s];
        if (cur == 0) {
          uint32_t prev = atomicCAS(&keys[s], 0u, k1);
          cur = prev == 0 ? k1 : prev;
        }
        if (cur == k1) {
          found = (int)s;
          break;
        }
        s = (s + 1) & mask;
      }
      if (found >= 0) {
        unsigned long long* d = reinterpret_cast<unsigned long long*>(vals + (int64_t)found * T.stride);
        atomicAdd(d, 1ull);
#pragma unroll
        for (int j = 0; j < NE; j++)
          if (j < nsum) atomicAdd(d + 1 + j, (unsigned long long)v[j]);
      } else {
        unsigned long long* g = reinterpret_cast<unsigned long long*>(T.data + key * T.stride);
        global_add(g, 1);
#pragma unroll
        for (int j = 0; j < NE; j++)
          if (j < nsum) global_add(g + 1 + j, v[j]);
      }
    }
  }

  // The COUNT of group `key` (for add() split in two: the caller then adds sum
  // j at at[1 + j]). Returns false for a key outside the domain (remembered or
  // latched as in add()). *lds tells whether `at` is in LDS (else the
  // group's global entry, where adds must be device atomics).
  __device__ __forceinline__ bool count(const AggTarget& T, int64_t key, unsigned long long** at, bool* lds) {
    if ((uint64_t)key >= (uint64_t)T.domain) {
      if (defer) bad = true;
      else latch_error(T.err, TQ_EDOMAIN);
      return false;
    }
    *lds = true;
    if (MODE == kDense) {
      *at = reinterpret_cast<unsigned long long*>(vals + key * T.stride);
    } else {
      uint32_t k1 = (uint32_t)key + 1u;
      uint32_t mask = (1u << T.log2hcap) - 1u;
      uint32_t s = ((uint32_t)key * 0x9E3779B1u) >> (32 - T.log2hcap);
      int found = -1;
      for (int i = 0; i < kHashProbes; i++) {
        uint32_t cur = keys[s];
        if (cur == 0) {
          uint32_t prev = atomicCAS(&keys[s], 0u, k1);
          cur = prev == 0 ? k1 : prev;
        }
        if (cur == k1) {
          found = (int)s;
          break;
        }
        s = (s + 1) & mask;
      }
      *lds = found >= 0;
      *at = *lds ? reinterpret_cast<unsigned long long*>(vals + (int64_t)found * T.stride)
                 : reinterpret_cast<unsigned long long*>(T.data + key * T.stride);
    }
    if (*lds) atomicAdd(*at, 1ull);
    else global_add(*at, 1);
    return true;
  }

  // Nullable states: group `key` (T.udomain: the NULL group; a key outside
  // [0, udomain] is remembered or latched as TQ_EDOMAIN), COUNT(*) += 1, and
  // for each sum j present in the row (bit j of `present`) SUM_j += v[j] and
  // COUNT_j += 1 (entries 1 + 2j and 2 + 2j).
  template <int NE>
  __device__ __forceinline__ void add_nullable(const AggTarget& T, int64_t key, const int64_t (&v)[NE],
                                               uint32_t present, int nsum) {
    unsigned long long* at;
    bool in_lds;
    if (!count(T, key, &at, &in_lds)) return;
#pragma unroll
    for (int j = 0; j < NE; j++) {
      if (j < nsum && ((present >> j) & 1u)) {
        if (in_lds) {
          atomicAdd(at + 1 + 2 * j, (unsigned long long)v[j]);
          atomicAdd(at + 2 + 2 * j, 1ull);
        } else {
          global_add(at + 1 + 2 * j, v[j]);
          global_add(at + 2 + 2 * j, 1);
        }
      }
    }
  }

  // Folds this workgroup's LDS partials into the global state.
  __device__ void flush(const AggTarget& T) {
    if (bad) latch_error(T.err, TQ_EDOMAIN);
    __syncthreads();
    if (MODE == kDense) {
      const int64_t entries = T.domain * T.stride;
      if (T.rows > 1) {
        int64_t* row = T.data + (int64_t)blockIdx.x * entries;
        for (int64_t e = threadIdx.x; e < entries; e += blockDim.x) row[e] += vals[e];
        // calls on one state are stream ordered, so one writer suffices
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          StateHeader* h = const_cast<StateHeader*>(T.hdr);
          if (h->used < (int64_t)gridDim.x) h->used = gridDim.x;
        }
      } else {
        for (int64_t k = threadIdx.x; k < T.domain; k += blockDim.x) {
          const int64_t* src = vals + k * T.stride;
          if (src[0] == 0) continue;
          unsigned long long* g = reinterpret_cast<unsigned long long*>(T.data + k * T.stride);
          for (int j = 0; j < T.stride; j++) global_add(g + j, src[j]);
        }
      }
    } else {
      int hcap = 1 << T.log2hcap;
      for (int s = threadIdx.x; s < hcap; s += blockDim.x) {
        uint32_t k1 = keys[s];
        if (k1 == 0) continue;
        const int64_t* src = vals + (int64_t)s * T.stride;
        unsigned long long* g = reinterpret_cast<unsigned long long*>(T.data + (int64_t)(k1 - 1) * T.stride);
        for (int j = 0; j < T.stride; j++) global_add(g + j, src[j]);
      }
    }
  }
};

// nullable: the state of tq_groupby_init_nullable (domain + 1 groups, 1 + 2 * nsum entries each).
tq_status make_target(void* d_state, int64_t domain, int32_t nsum, AggTarget* T, AggMode* mode, size_t* lds,
                      bool nullable = false);
int agg_grid(int64_t n);

// Smallest supported sum-count bucket >= ne (the aggregating kernels are
// instantiated per bucket so that only live sums occupy registers).
inline int ne_bucket(int ne) { return ne <= 1 ? 1 : ne <= 2 ? 2 : 6; }

#define TQ_DISPATCH_AGG(mode, ncol, ne, MODEV, NCV, NEV, ...)                           \
  do {                                                                                  \
    auto run_ = [&](auto mode_c, auto nc_c, auto ne_c) {                                \
      constexpr int MODEV = decltype(mode_c)::value;                                    \
      constexpr int NCV = decltype(nc_c)::value;                                        \
      constexpr int NEV = decltype(ne_c)::value;                                        \
      __VA_ARGS__;                                                                      \
    };                                                                                  \
    auto ne_ = [&](auto m_c, auto n_c) {                                                \
      switch (::tq::ne_bucket(ne)) {                                                    \
        case 1: run_(m_c, n_c, std::integral_constant<int, 1>{}); break;                \
        case 2: run_(m_c, n_c, std::integral_constant<int, 2>{}); break;                \
        default: run_(m_c, n_c, std::integral_constant<int, 6>{}); break;               \
      }                                                                                 \
    };                                                                                  \
    auto nc_ = [&](auto m_c) {                                                          \
      switch (::tq::nc_bucket(ncol)) {                                                  \
        case 1: case 2: ne_(m_c, std::integral_constant<int, 2>{}); break;              \
        case 4: ne_(m_c, std::integral_constant<int, 4>{}); break;                      \
        default: ne_(m_c, std::integral_constant<int, 8>{}); break;                     \
      }                                                                                 \
    };                                                                                  \
    if ((mode) == ::tq::kDense) nc_(std::integral_constant<int, ::tq::kDense>{});       \
    else nc_(std::integral_constant<int, ::tq::kHash>{});                               \
  } while (0)

}  // namespace tq
