// Per-workgroup group-by partials in LDS, flushed to a replicated global state.
//
// Three modes, chosen on the host from the key domain and the entry width:
//   kDense   the whole domain fits in LDS: direct-indexed int64 partials
//   kHash    an LDS open-addressing table of hot keys (Zipf-skewed groups stay
//            on chip); rows whose key finds no LDS slot within a few probes go
//            straight to global atomics
//   kGlobal  no LDS; every row is a global atomic
// A global entry (key k, value j) lives at data[r * domain * stride + k * stride + j]
// for replica r = blockIdx.x mod replicas; finalization sums the replicas.
// Value 0 of every entry is COUNT, values 1..nsum are the SUMs.
#pragma once

#include "common.h"

namespace tq {

enum AggMode { kDense = 0, kHash = 1, kGlobal = 2 };

constexpr int kLdsAggBytes = 32 * 1024;
constexpr int kHashProbes = 8;

struct AggTarget {
  const StateHeader* hdr;
  int64_t* data;    // global replicas
  int32_t* err;     // latched error of the state
  int64_t domain;
  int32_t stride;   // 1 + nsum
  int32_t replicas;
  int32_t log2hcap; // kHash: LDS slots = 1 << log2hcap
};

// The launch parameters must describe the state the buffer was initialised
// with; otherwise the kernel writes nothing (tq_check then reports the error).
__device__ __forceinline__ bool state_matches(const AggTarget& T) {
  const StateHeader* h = T.hdr;
  if (h->magic != kStateMagic) return false;
  if (h->domain != T.domain || h->nsum != T.stride - 1 || h->replicas != T.replicas) {
    if (threadIdx.x == 0) latch_error(T.err, TQ_EINVAL);
    return false;
  }
  return true;
}

// Host: pick the mode and the dynamic LDS size for a state.
inline AggMode agg_mode(int64_t domain, int stride, int* log2hcap, size_t* lds_bytes) {
  if (domain * stride * 8 <= kLdsAggBytes) {
    *log2hcap = 0;
    *lds_bytes = (size_t)domain * stride * 8;
    return kDense;
  }
  int per_slot = 4 + stride * 8;
  int l = 0;
  while ((size_t)(2 << l) * per_slot <= (size_t)kLdsAggBytes && l < 14) l++;
  if (l >= 6) {
    *log2hcap = l;
    *lds_bytes = ((size_t)(1 << l) * 4 + 15) / 16 * 16 + (size_t)(1 << l) * stride * 8;
    return kHash;
  }
  *log2hcap = 0;
  *lds_bytes = 0;
  return kGlobal;
}

inline int choose_replicas(int64_t domain, int stride) {
  int64_t e = domain * stride;
  int r = 1;
  while (r < 32 && (int64_t)r * 2 * e <= 16384) r *= 2;
  return r;
}

template <int MODE>
struct LdsAgg {
  int64_t* vals;   // kDense: [domain][stride]; kHash: [hcap][stride]
  uint32_t* keys;  // kHash: key + 1, 0 = empty

  __device__ void init(const AggTarget& T, char* smem) {
    if (MODE == kDense) {
      vals = reinterpret_cast<int64_t*>(smem);
      for (int64_t i = threadIdx.x; i < T.domain * T.stride; i += blockDim.x) vals[i] = 0;
    } else if (MODE == kHash) {
      int hcap = 1 << T.log2hcap;
      keys = reinterpret_cast<uint32_t*>(smem);
      vals = reinterpret_cast<int64_t*>(smem + (((size_t)hcap * 4 + 15) / 16 * 16));
      for (int i = threadIdx.x; i < hcap; i += blockDim.x) keys[i] = 0;
      for (int i = threadIdx.x; i < hcap * T.stride; i += blockDim.x) vals[i] = 0;
    }
  }

  __device__ __forceinline__ int64_t* global_entry(const AggTarget& T, int64_t key) const {
    int r = blockIdx.x & (T.replicas - 1);
    return T.data + (int64_t)r * T.domain * T.stride + key * T.stride;
  }

  // Adds COUNT 1 and the nsum values v[0..nsum) to group `key`.
  __device__ __forceinline__ void add(const AggTarget& T, int64_t key, const int64_t (&v)[TQ_MAX_SUMS], int nsum) {
    if ((uint64_t)key >= (uint64_t)T.domain) {
      latch_error(T.err, TQ_EDOMAIN);
      return;
    }
    int64_t* dst = nullptr;
    if (MODE == kDense) {
      dst = vals + key * T.stride;
    } else if (MODE == kHash) {
      uint32_t k1 = (uint32_t)key + 1u;
      uint32_t mask = (1u << T.log2hcap) - 1u;
      uint32_t s = ((uint32_t)key * 0x9E3779B1u) >> (32 - T.log2hcap);
      for (int i = 0; i < kHashProbes; i++) {
        uint32_t cur = keys[s];
        if (cur == 0) cur = atomicCAS(&keys[s], 0u, k1), cur = cur == 0 ? k1 : cur;
        if (cur == k1) {
          dst = vals + (int64_t)s * T.stride;
          break;
        }
        s = (s + 1) & mask;
      }
    }
    if (dst == nullptr) dst = global_entry(T, key);  // kGlobal, or no LDS slot found
    atomicAdd(reinterpret_cast<unsigned long long*>(dst), 1ull);
#pragma unroll
    for (int j = 0; j < TQ_MAX_SUMS; j++)
      if (j < nsum) atomicAdd(reinterpret_cast<unsigned long long*>(dst + 1 + j), (unsigned long long)v[j]);
  }

  // Adds the LDS partials of this workgroup to the global state.
  __device__ void flush(const AggTarget& T) {
    __syncthreads();
    if (MODE == kDense) {
      for (int64_t k = threadIdx.x; k < T.domain; k += blockDim.x) {
        const int64_t* src = vals + k * T.stride;
        if (src[0] == 0) continue;
        int64_t* dst = global_entry(T, k);
        for (int j = 0; j < T.stride; j++) atomicAdd(reinterpret_cast<unsigned long long*>(dst + j), (unsigned long long)src[j]);
      }
    } else if (MODE == kHash) {
      int hcap = 1 << T.log2hcap;
      for (int s = threadIdx.x; s < hcap; s += blockDim.x) {
        uint32_t k1 = keys[s];
        if (k1 == 0) continue;
        const int64_t* src = vals + (int64_t)s * T.stride;
        int64_t* dst = global_entry(T, (int64_t)(k1 - 1));
        for (int j = 0; j < T.stride; j++) atomicAdd(reinterpret_cast<unsigned long long*>(dst + j), (unsigned long long)src[j]);
      }
    }
  }
};

}  // namespace tq
