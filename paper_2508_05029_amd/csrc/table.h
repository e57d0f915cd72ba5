// Device-side operations on the bucketized open-addressing join table, shared
// by the stand-alone join kernels and the batched persistent kernel.
//
// Open addressing with linear probing over buckets of 8 slots: a key's home
// bucket comes from the high bits of its 64-bit multiplicative hash, its tag
// from the low 16 bits (0 means empty). Inserts fill a bucket's free slots,
// then move to the next bucket; a probe reads the 8 tags of a bucket with one
// 16-byte load and stops at the first bucket that has an empty slot.
#pragma once

#include "common.h"

namespace tq {

// Bits j (0..7) of the result: tag j of the bucket equals t.
__device__ __forceinline__ uint32_t tag_match(const v4i32& w, uint32_t t) {
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    uint32_t x = (uint32_t)w[q];
    m |= (uint32_t)((x & 0xffffu) == t) << (2 * q);
    m |= (uint32_t)((x >> 16) == t) << (2 * q + 1);
  }
  return m;
}

// Whether some tag of the bucket is 0 (a free slot). Per 32-bit word of two
// tags, (x - 0x00010001) & ~x has a lane's top bit set exactly when that lane
// is the lowest zero one (a borrow leaves only a zero lane); as a yes/no over
// the word the test is exact, in two instructions instead of a mask's eight.
__device__ __forceinline__ bool has_empty(const v4i32& w) {
  uint32_t a = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const uint32_t x = (uint32_t)w[q];
    a |= (x - 0x00010001u) & ~x;
  }
  return (a & 0x80008000u) != 0u;
}

__device__ __forceinline__ uint32_t word_of(const v4i32& w, int q) {
  uint32_t r = (uint32_t)w[0];
  r = q == 1 ? (uint32_t)w[1] : r;
  r = q == 2 ? (uint32_t)w[2] : r;
  r = q == 3 ? (uint32_t)w[3] : r;
  return r;
}

__device__ __forceinline__ void set_word(v4i32& w, int q, uint32_t v) {
  w[0] = q == 0 ? (int)v : w[0];
  w[1] = q == 1 ? (int)v : w[1];
  w[2] = q == 2 ? (int)v : w[2];
  w[3] = q == 3 ? (int)v : w[3];
}

// Inserts up to R (key, payload) rows of one lane (those with pend[i] set).
// Each round issues at most one CAS per row, for the first free slot at or
// after the row's start slot (hash bits, so that inserters into one bucket
// spread over its slots) in the row's view of its bucket. The view starts as
// "empty" and is corrected by the word a failed CAS returns, so every round
// claims a slot, learns of a newly taken one, or moves to the next bucket.
template <int R>
__device__ __forceinline__ void table_insert(uint32_t* words, v2i64* slots, int log2cap, int skip, bool (&pend)[R],
                                             const int64_t (&k)[R], const int64_t (&pay)[R]) {
  const int64_t cap = (int64_t)1 << log2cap, bmask = (cap >> kLog2Bucket) - 1;
  int64_t b[R];
  uint32_t tg[R];
  int st[R];
  v4i32 w[R];
#pragma unroll
  for (int i = 0; i < R; i++) {
    uint64_t hh = mulhash(k[i]);
    b[i] = (int64_t)bucket_of(hh, skip, log2cap - kLog2Bucket);
    tg[i] = hash_tag(hh);
    st[i] = (int)(hh >> 16) & (kBucket - 1);
    w[i] = v4i32{0, 0, 0, 0};
  }
  for (int64_t round = 0; round < 2 * cap + 8; round++) {
    uint32_t expect[R], prev[R];
    int slot[R];
    bool tried[R];
#pragma unroll
    for (int i = 0; i < R; i++) {
      tried[i] = false;
      slot[i] = 0;
      expect[i] = 0;
      prev[i] = 0;
      if (!pend[i]) continue;
      uint32_t zero = tag_match(w[i], 0u);
      if (zero == 0u) {  // bucket full: linear probing moves to the next bucket
        b[i] = (b[i] + 1) & bmask;
        w[i] = v4i32{0, 0, 0, 0};
        continue;
      }
      uint32_t rot = ((zero >> st[i]) | (zero << (kBucket - st[i]))) & 0xffu;
      slot[i] = (__builtin_ctz(rot) + st[i]) & (kBucket - 1);
      int q = slot[i] >> 1;
      expect[i] = word_of(w[i], q);
      uint32_t desired = expect[i] | (tg[i] << ((slot[i] & 1) * 16));
      prev[i] = atomicCAS(&words[b[i] * 4 + q], expect[i], desired);
      tried[i] = true;
    }
    bool more = false;
#pragma unroll
    for (int i = 0; i < R; i++) {
      if (tried[i]) {
        if (prev[i] == expect[i]) {
          v2i64 kv = {k[i], pay[i]};
          slots[b[i] * kBucket + slot[i]] = kv;
          pend[i] = false;
        } else {
          set_word(w[i], slot[i] >> 1, prev[i]);
        }
      }
      more = more || pend[i];
    }
    if (!more) break;
  }
}

// Bucket after b in its chain: linear probing that wraps inside b's region of
// 2^log2g buckets (the whole table when log2g = log2 of the bucket count).
__device__ __forceinline__ int64_t next_bucket(int64_t b, int64_t gmask) { return (b & ~gmask) | ((b + 1) & gmask); }

struct Probe {
  const v4i32* groups;
  const v2i64* slots;
  int64_t bmask, gmask, cap;
  int log2b, skip;
  bool unique;
  uint32_t sel = 0;  // the build's flags when it kept one hash partition (a probe row of another matches nothing)

  __device__ __forceinline__ void setup(const TableHeader* h) {
    TableHeader* t = const_cast<TableHeader*>(h);
    const bool alt = h->alt != 0;  // a fallback build used the scratch arrays
    setup(alt ? scratch_alt_tags(t, h->cap_max) : table_tags(t),
          alt ? scratch_rows(t, h->cap_max) : table_slots(t, h->cap_max), h->log2cap, h->skip,
          (h->flags & TQ_UNIQUE_KEYS) != 0, h->log2g);
    sel = h->flags & TQ_SELECT_PARTITION ? h->flags : 0u;
  }

  __device__ __forceinline__ bool selected(uint64_t hh) const { return in_partition(hh, skip, sel); }

  // log2g < 0: one region spanning the table
  __device__ __forceinline__ void setup(const uint32_t* words, const int64_t* slot_base, int log2cap, int skip_bits,
                                        bool unique_keys, int log2g = -1) {
    log2b = log2cap - kLog2Bucket;
    skip = skip_bits;
    unique = unique_keys;
    cap = (int64_t)1 << log2cap;
    bmask = ((int64_t)1 << log2b) - 1;
    gmask = (log2g < 0 || log2g > log2b) ? bmask : ((int64_t)1 << log2g) - 1;
    groups = reinterpret_cast<const v4i32*>(words);
    slots = reinterpret_cast<const v2i64*>(slot_base);
  }

  // Walks the chains of one lane's rows in lockstep. Each round checks one
  // tag-matching slot per row (or moves the row to its next bucket) and calls
  // on_round(hit, payload): hit[i] is set when row i matched in this round (a
  // row can match again in later rounds unless the build keys are unique).
  template <int R, typename F>
  __device__ __forceinline__ void walk(const bool (&ok)[R], const int64_t (&k)[R], F&& on_round) const {
    walk(ok, k, on_round, [] {});
  }

  // As above; `issued()` runs once, right after the first tag loads are issued
  // (a caller prefetches its next rows there, so that the wait for the tags
  // does not also wait for the prefetch).
  template <int R, typename F, typename G>
  __device__ __forceinline__ void walk(const bool (&ok)[R], const int64_t (&k)[R], F&& on_round, G&& issued) const {
    int64_t b[R];
    uint32_t tg[R], m[R];
    bool act[R], empty[R], load[R];
#pragma unroll
    for (int i = 0; i < R; i++) {
      uint64_t hh = mulhash(k[i]);
      b[i] = (int64_t)bucket_of(hh, skip, log2b);
      tg[i] = hash_tag(hh);
      act[i] = ok[i] && selected(hh);
      load[i] = true;
      m[i] = 0;
      empty[i] = false;
    }
    for (int64_t round = 0; round < 2 * cap + 8; round++) {
      v4i32 w[R];
#pragma unroll
      for (int i = 0; i < R; i++)
        if (act[i] && load[i]) w[i] = groups[b[i]];
      if (round == 0) issued();
#pragma unroll
      for (int i = 0; i < R; i++) {
        if (act[i] && load[i]) {
          m[i] = tag_match(w[i], tg[i]);
          empty[i] = has_empty(w[i]);
          load[i] = false;
        }
      }
      v2i64 kv[R];
      bool cand[R], hit[R];
      int64_t pay[R];
#pragma unroll
      for (int i = 0; i < R; i++) {
        cand[i] = act[i] && m[i] != 0u;
        int j = cand[i] ? __builtin_ctz(m[i]) : 0;
        kv[i] = cand[i] ? slots[b[i] * kBucket + j] : v2i64{0, 0};
        m[i] &= m[i] - 1u;
      }
#pragma unroll
      for (int i = 0; i < R; i++) {
        hit[i] = cand[i] && kv[i].x == k[i];
        pay[i] = kv[i].y;
      }
      on_round(hit, pay);
      bool more = false;
#pragma unroll
      for (int i = 0; i < R; i++) {
        if (!act[i]) continue;
        if (hit[i] && unique) act[i] = false;
        else if (m[i] == 0u) {
          if (empty[i]) act[i] = false;  // an empty slot ends the chain
          else {
            b[i] = next_bucket(b[i], gmask);
            load[i] = true;
          }
        }
        more = more || act[i];
      }
      if (!more) break;
    }
  }
};

}  // namespace tq
