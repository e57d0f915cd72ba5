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
constexpr int kMaxCountBlocks = 1024;  // build count blocks (their partials are summed by every insert block)

__host__ __device__ inline int log2cap_for(int64_t rows, double lf) {
  double need = ceil((double)rows / lf);
  int l = 6;
  while (l < 62 && (double)((int64_t)1 << l) < need) l++;
  return l;
}

__host__ __device__ inline size_t table_bytes_for(int64_t cap) {
  return kHeaderBytes + (size_t)kMaxPartBlocks * 8 + table_tag_bytes(cap) + (size_t)cap * 16 + scratch_bytes(cap);
}

// The capacity rule as integer thresholds, for kernels that apply it to a
// device-side count: t[l] is the largest row count whose capacity
// (log2cap_for) is at most 2^l, found with the same double arithmetic.
struct CapRule {
  int64_t t[62];
};
static CapRule cap_rule(double lf) {
  CapRule R;
  for (int l = 0; l < 62; l++) {
    int64_t lo = -1, hi = (int64_t)1 << 61;  // log2cap_for(lo) <= l < log2cap_for(hi)
    if (l < 6) {
      R.t[l] = -1;
      continue;
    }
    while (hi - lo > 1) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (log2cap_for(mid, lf) <= l) lo = mid;
      else hi = mid;
    }
    R.t[l] = lo;
  }
  return R;
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

// A build row's admission under NULLs (nulls: some column carries a
// validity bitmap): the filter (a predicate over NULL is not true) and a
// present key. Without NULLs, the filter alone.
template <int NC, int R>
__device__ __forceinline__ bool build_row_ok(const RowPlan& P, const int64_t (&v)[NC][R], int i, int64_t r,
                                             const uint8_t* key_valid, bool nulls) {
  if (!nulls) return eval_preds<NC>(P, v, i);
  return (!key_valid || bit_at(key_valid, r)) && eval_preds_present<NC>(P, v, i, row_present<NC>(P, r));
}

// The stored payload: INT64_MIN stands for a NULL one.
__device__ __forceinline__ int64_t stored_payload(const DCol& pc, int64_t r, int64_t pay) {
  return pc.valid && !bit_at(pc.valid, r) ? INT64_MIN : pay;
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
  h->log2g = 6 - kLog2Bucket;
  h->regions = 0;
  h->alt = 0;
  h->ovf = 0;
  h->bloom_log2w = 0;
}

// ------------------------------------------------------------------ build

// Pass 1: the filtered row count of each block's contiguous range (into the
// table's partial area), and the whole tag array cleared (the capacity the
// rows need is only known once every block has counted).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_build_count(RowPlan P, const int64_t* keys, int64_t n, int64_t per,
                                                        TableHeader* h, int64_t cap_max, int count, int skip,
                                                        uint32_t flags, const uint8_t* key_valid) {
  __shared__ int64_t ws[kBlock / kWave];
  if (h->magic != kTableMagic) return;  // never initialised: the insert kernel does nothing either
  // a new build: an error latched by an earlier build into this buffer no longer applies
  if (blockIdx.x == 0 && threadIdx.x == 0) h->err = 0;
  v4i32* tags = reinterpret_cast<v4i32*>(table_tags(h));
  const v4i32 z = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (cap_max >> kLog2Bucket);
       i += (int64_t)gridDim.x * blockDim.x)
    tags[i] = z;
  if (!count) return;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  int64_t c = 0;
  const DCol kc = {keys, 8};
  const bool sel = (flags & TQ_SELECT_PARTITION) != 0;
  const bool nulls = P.null_cols != 0 || key_valid != nullptr;
  for (int64_t r0 = lo + threadIdx.x * kRows; r0 < hi; r0 += kChunk) {
    int64_t v[NC][kRows], k[kRows];
    load_rows<NC>(P, r0, r0 + kRows <= hi, hi, v);
    if (sel) load4(kc, r0, r0 + kRows <= hi, hi, k);
#pragma unroll
    for (int i = 0; i < kRows; i++)
      c += (r0 + i < hi) && build_row_ok<NC>(P, v, i, r0 + i, key_valid, nulls) &&
           (!sel || in_partition(mulhash(k[i]), skip, flags));
  }
  int64_t t = block_sum(c, ws);
  if (threadIdx.x == 0) table_partials(h)[blockIdx.x] = t;
}

// Pass 2: every block fixes the capacity from the row count (host-given, or
// the sum of the per-block counts; block 0 records it in the header) and
// inserts its rows.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_build_insert(RowPlan P, const int64_t* keys, DCol payload, int64_t n,
                                                         TableHeader* h, int64_t cap_max, int64_t n_host, int nblk,
                                                         double lf, int skip, uint32_t flags,
                                                         const uint8_t* key_valid) {
  __shared__ int64_t ws[kBlock / kWave];
  if (h->magic != kTableMagic) return;
  int64_t rows = n_host;
  if (n_host < 0) {
    int64_t c = 0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) c += table_partials(h)[b];
    rows = block_sum(c, ws);
  }
  int l = log2cap_for(rows, lf);
  const bool full = ((int64_t)1 << l) > cap_max;
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
    h->log2g = l - kLog2Bucket;
    h->regions = 0;
    h->alt = 0;
    h->bloom_log2w = 0;
    if (full) latch_error(&h->err, TQ_EFULL);
  }
  if (full) return;  // does not fit: TQ_EFULL is latched, nothing is inserted
  uint32_t* words = table_tags(h);
  v2i64* slots = reinterpret_cast<v2i64*>(table_slots(h, cap_max));
  const DCol kc = {keys, 8};
  const bool nulls = P.null_cols != 0 || key_valid != nullptr;
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    const bool fullrow = r0 + kRows <= n;
    int64_t v[NC][kRows], k[kRows], pay[kRows];
    bool pend[kRows];
    load_rows<NC>(P, r0, fullrow, n, v);
    load4(kc, r0, fullrow, n, k);
    load4(payload, r0, fullrow, n, pay);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      pend[i] = (r0 + i < n) && build_row_ok<NC>(P, v, i, r0 + i, key_valid, nulls) &&
                in_partition(mulhash(k[i]), skip, flags);
      if (pend[i]) pay[i] = stored_payload(payload, r0 + i, pay[i]);
    }
    table_insert<kRows>(words, slots, l, skip, pend, k, pay);
  }
}

// ------------------------------------------------------------------ region build
//
// The common case of a build that fits: no global atomics per row. Each table
// region (the buckets that share the top kLog2Bins bits of their index, with
// linear probing wrapping inside the region) is filled in LDS by one
// workgroup and written out whole. Three launches, so that each reads what
// the previous one wrote without any wait between workgroups:
//   k_build_part     each block filters and hashes its kPartRows rows and
//                    groups the passing ones by region in its own segment of
//                    the scratch area, recording (offset, count) per region.
//   k_build_regions  every workgroup sums the block counts and fixes the
//                    capacity; workgroup j gathers region j's rows from every
//                    segment, inserts them into an LDS copy of the region and
//                    stores its tags and slots. A region whose rows would not
//                    leave it a free slot (a probe's walk ends at one), or a
//                    capacity outside the LDS range, sets the overflow flag.
//   k_build_fallback nothing unless the flag is set; then the global CAS
//                    insert of every row into the scratch's alternate tags and
//                    slots (cleared by the previous launch), which the header
//                    then names as the arrays in use.

constexpr int kFinBlock = 1024;
constexpr int kMaxRegionSlots = 2048;  // LDS region: 4 KiB of tags + 32 KiB of slots
static_assert(kFinBlock == kMaxRegionSlots / 2, "one thread clears one LDS tag word");
constexpr int kMinRegionLog2Cap = kLog2Bucket + kLog2Bins;  // a region of at least one bucket
constexpr int kMaxRegionLog2Cap = 11 + kLog2Bins;            // at most kMaxRegionSlots slots
constexpr int kMaxPassLog2Cap = kMaxRegionLog2Cap + 4;        // regions of up to 16 LDS domains
constexpr int kMaxSubs = 1 << (kMaxPassLog2Cap - kMaxRegionLog2Cap);

template <int NC>
__global__ __launch_bounds__(kPartBlock) void k_build_part(RowPlan P, const int64_t* keys, DCol payload, int64_t n,
                                                          TableHeader* h, int64_t cap_max, int skip, uint32_t flags,
                                                          const uint8_t* key_valid) {
  __shared__ uint32_t hist[kRegionBins];
  __shared__ uint32_t loc[kRegionBins];
  __shared__ int64_t ws[kPartBlock / kWave];
  const int tid = threadIdx.x;
  // kPartSub groups of kRows consecutive rows per thread, the groups a block
  // width apart: every load of a group is issued before any row is hashed
  int64_t v[kPartSub][NC][kRows], k[kPartSub][kRows], pay[kPartSub][kRows];
  const DCol kc = {keys, 8};
#pragma unroll
  for (int c = 0; c < kPartSub; c++) {
    const int64_t r0 = (int64_t)blockIdx.x * kPartRows + ((int64_t)c * kPartBlock + tid) * kRows;
    const bool full = r0 + kRows <= n;
    load_rows<NC>(P, r0, full, n, v[c]);
    load4(kc, r0, full, n, k[c]);
    load4(payload, r0, full, n, pay[c]);
  }
  if (h->magic != kTableMagic) return;
  if (blockIdx.x == 0 && tid == 0) {
    h->ovf = 0;  // the previous build's fallback has finished with it
    h->err = 0;  // and an error it latched no longer applies
  }
  if (tid < kRegionBins) hist[tid] = 0;
  __syncthreads();
  const bool nulls = P.null_cols != 0 || key_valid != nullptr;
  bool ok[kPartSub][kRows];
  uint32_t bin[kPartSub][kRows], rank[kPartSub][kRows];
#pragma unroll
  for (int c = 0; c < kPartSub; c++) {
    const int64_t r0 = (int64_t)blockIdx.x * kPartRows + ((int64_t)c * kPartBlock + tid) * kRows;
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      const uint64_t hh = mulhash(k[c][i]);
      ok[c][i] = (r0 + i < n) && build_row_ok<NC>(P, v[c], i, r0 + i, key_valid, nulls) &&
                 in_partition(hh, skip, flags);
      if (ok[c][i]) pay[c][i] = stored_payload(payload, r0 + i, pay[c][i]);
      bin[c][i] = (uint32_t)((hh << skip) >> (64 - kLog2Bins));
      rank[c][i] = ok[c][i] ? atomicAdd(&hist[bin[c][i]], 1u) : 0u;
    }
  }
  __syncthreads();
  const uint32_t cnt = tid < kRegionBins ? hist[tid] : 0u;
  int64_t excl;
  const int64_t total = block_excl_scan((int64_t)cnt, &excl, ws);
  if (tid < kRegionBins) {
    loc[tid] = (uint32_t)excl;
    scratch_meta(h, cap_max)[(size_t)blockIdx.x * kMetaStride + tid] = ((uint32_t)excl << 16) | cnt;
  }
  if (tid == 0) scratch_block_rows(h, cap_max)[blockIdx.x] = (int32_t)total;
  __syncthreads();
  v2i64* seg = reinterpret_cast<v2i64*>(scratch_rows(h, cap_max)) + (size_t)blockIdx.x * kPartRows;
#pragma unroll
  for (int c = 0; c < kPartSub; c++)
#pragma unroll
    for (int i = 0; i < kRows; i++)
      if (ok[c][i]) seg[loc[bin[c][i]] + rank[c][i]] = v2i64{k[c][i], pay[c][i]};
}

// The region a k_build_regions workgroup fills. Workgroups are dealt to the
// eight XCDs in turn (workgroup i to XCD i mod 8), so workgroup i takes region
// (i mod 8) * 32 + i / 8: each XCD fills 32 adjacent regions, whose counts in
// a block's metadata row share one cache line and whose rows lie together in
// each block's segment, so that each line is fetched into one XCD's L2, not
// into up to eight.
__device__ __forceinline__ int region_of_workgroup(int i) {
  constexpr int kXcds = 8, kPer = kRegionBins / kXcds;
  return (i % kXcds) * kPer + i / kXcds;
}

__global__ __launch_bounds__(kFinBlock) void k_build_regions(TableHeader* h, int64_t cap_max, int nblk, double lf,
                                                            int skip, uint32_t flags, CapRule rule) {
  __shared__ uint32_t ltag[kMaxRegionSlots / 2];
  __shared__ v2i64 lslot[kMaxRegionSlots];
  __shared__ int64_t ws[2 * kFinBlock / kWave];
  __shared__ uint32_t lbloom[kGBloomWordsMax / kRegionBins];
  __shared__ uint32_t sub_cnt[kMaxSubs], sub_fill[kMaxSubs], sub_off[kMaxSubs + 1];
  const int j = region_of_workgroup(blockIdx.x), tid = threadIdx.x;
  const uint32_t* meta = scratch_meta(h, cap_max) + j;  // region j's counts, block b at meta[b * kMetaStride]
  // the loads go out first (the scratch lies inside the caller's buffer
  // whatever the header holds), then the LDS copy is cleared while they fly
  const int32_t* brows = scratch_block_rows(h, cap_max);
  int64_t rb = 0, cj = 0;
  uint32_t m0 = 0;
  for (int b = tid; b < nblk; b += kFinBlock) {
    const uint32_t m = meta[(size_t)b * kMetaStride];
    rb += brows[b];
    cj += m & 0xffffu;
    if (b == tid) m0 = m;
  }
  ltag[tid] = 0u;  // kFinBlock == kMaxRegionSlots / 2
  for (int i = tid; i < kGBloomWordsMax / kRegionBins; i += kFinBlock) lbloom[i] = 0u;
  if (tid < kMaxSubs) sub_cnt[tid] = sub_fill[tid] = 0u;
  if (h->magic != kTableMagic) return;
  int64_t rows = rb, mine = cj;  // all rows; rows of region j
  block_sum2(&rows, &mine, ws);
  rows = ((int64_t)__builtin_amdgcn_readfirstlane((int)(rows >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)rows);  // uniform: scalar from here
  int l = 6;  // log2cap_for(rows, lf)
  while (l < 62 && rows > rule.t[l]) l++;
  const bool too_big = ((int64_t)1 << l) > cap_max;
  if (too_big) {
    l = 6;
    while (((int64_t)1 << (l + 1)) <= cap_max) l++;
  }
  // Up to kMaxRegionLog2Cap a region is one LDS domain, filled in one pass.
  // Up to kMaxPassLog2Cap it is 2^(l - kMaxRegionLog2Cap) domains of
  // kMaxRegionSlots slots, filled one after the other (linear probing wraps
  // inside a domain either way).
  const bool in_range = l >= kMinRegionLog2Cap && l <= kMaxPassLog2Cap;
  const bool multi = l > kMaxRegionLog2Cap;
  const int sub_log2 = multi ? l - kMaxRegionLog2Cap : 0;
  const int64_t region_slots = in_range ? (int64_t)1 << (l - kLog2Bins) : 0;
  const bool fits = in_range && (multi || mine <= region_slots - std::max<int64_t>(1, region_slots / 8));
  // Bloom words (log2) for this capacity: bloom_words_max(2^l), two bits per
  // slot (every region-built capacity has its filter)
  const int log2w = in_range ? std::max(l - 4, kLog2Bins + 1) : 0;
  static_assert(kBloomWordsMax == 1 << kLog2BloomWordsMax && kRegionBins == 1 << kLog2Bins &&
                    kGBloomWordsMax == 1 << kLog2GBloomWordsMax && kMaxPassLog2Cap - 4 <= kLog2GBloomWordsMax,
                "bloom size rule");
  const int log2g = std::min(l, kMaxRegionLog2Cap) - kLog2Bucket - kLog2Bins;  // buckets per domain
  if (blockIdx.x == 0 && tid == 0) {
    h->cap_max = cap_max;
    h->n = rows;
    h->log2cap = l;
    h->skip = skip;
    h->flags = flags;
    h->lf = lf;
    h->log2g = log2g;
    h->regions = 1;
    h->alt = 0;
    h->bloom_log2w = log2w;
    if (too_big) latch_error(&h->err, TQ_EFULL);
  }
  if (too_big) return;  // TQ_EFULL is latched: nothing is inserted
  // the alternate tags, for a fallback insert (its launch decides)
  {
    v4i32* at = reinterpret_cast<v4i32*>(scratch_alt_tags(h, cap_max));
    const v4i32 z = {0, 0, 0, 0};
    const int64_t groups = (int64_t)1 << (l - kLog2Bucket);
    for (int64_t i = (int64_t)blockIdx.x * kFinBlock + tid; i < groups; i += (int64_t)gridDim.x * kFinBlock) at[i] = z;
  }
  if (!fits) {
    if (tid == 0) atomicOr(&h->ovf, 1);
    return;
  }
  const int gmask = (1 << log2g) - 1, nslot = kBucket << log2g;
  const int nbw = log2w ? 1 << (log2w - kLog2Bins) : 0;  // Bloom words of this region
  const v2i64* seg = reinterpret_cast<const v2i64*>(scratch_rows(h, cap_max));
  bool stuck = false;
  const int lane = tid & (kWave - 1);
  // Calls body(kv) for every row of region j: each wave takes 64 source
  // blocks at a time and spreads their rows of region j over its lanes (a wave
  // scan of the counts, then a search over the lanes by shuffles), so that
  // every lane loads one row at a time.
  auto each_row = [&](auto&& body) {
    for (int b0 = tid - lane; b0 < nblk; b0 += kFinBlock) {
      const int b = b0 + lane;
      const uint32_t m = b < nblk ? (b0 == tid - lane && b == tid ? m0 : meta[(size_t)b * kMetaStride]) : 0u;
      uint32_t total;
      const uint32_t excl = wave_excl_scan(m & 0xffffu, &total);
      const int64_t first = (int64_t)b * kPartRows + (m >> 16);  // this lane's first row in the segments
      // (every lane stays in the loop for the shuffles; only the row work is guarded)
      for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
        const uint32_t i = i0 + lane;
        int s = 0;  // the last lane whose rows start at or before i
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1)
          if ((uint32_t)__shfl(excl, s + step, kWave) <= i) s += step;
        const int64_t at = ((int64_t)__shfl((int)(first >> 32), s, kWave) << 32) |
                           (uint32_t)__shfl((int)(uint32_t)first, s, kWave);
        const uint32_t e_s = (uint32_t)__shfl(excl, s, kWave);
        if (i >= total) continue;
        body(seg[at + (i - e_s)]);
      }
    }
  };
  // Inserts a row into the LDS domain (its bucket's low log2g bits).
  auto insert = [&](const v2i64& kv, uint64_t hh) {
    int bl = (int)(bucket_of(hh, skip, l - kLog2Bucket) & (uint64_t)gmask);
    const uint32_t tg = hash_tag(hh);
    const int st = (int)(hh >> 16) & (kBucket - 1);
    // the domain keeps a free slot, so the walk finds one; the bound only
    // guards against a broken invariant
    bool done = false;
    for (int it = 0; it < 4 * nslot + 64 && !done; it++) {
      uint32_t w[4], zero = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        w[q] = ltag[bl * 4 + q];
        zero |= (uint32_t)((w[q] & 0xffffu) == 0u) << (2 * q);
        zero |= (uint32_t)((w[q] >> 16) == 0u) << (2 * q + 1);
      }
      if (zero == 0u) {
        bl = (bl + 1) & gmask;
        continue;
      }
      const uint32_t rot = ((zero >> st) | (zero << (kBucket - st))) & 0xffu;
      const int slot = (__builtin_ctz(rot) + st) & (kBucket - 1);
      const int q = slot >> 1;
      uint32_t cur = w[0];
      cur = q == 1 ? w[1] : cur;
      cur = q == 2 ? w[2] : cur;
      cur = q == 3 ? w[3] : cur;
      if (atomicCAS(&ltag[bl * 4 + q], cur, cur | (tg << ((slot & 1) * 16))) == cur) {
        lslot[bl * kBucket + slot] = kv;
        done = true;
      }
    }
    stuck = stuck || !done;
  };
  auto add_bloom = [&](uint64_t hh) {
    if (nbw) atomicOr(&lbloom[bloom_word(hh, skip, log2w) & (uint32_t)(nbw - 1)], bloom_bits(hh, log2w));
  };
  // Writes LDS domain d (of the whole table) out.
  auto write_domain = [&](int64_t d) {
    uint32_t* gw = table_tags(h) + ((size_t)d << log2g) * 4;
    for (int i = tid; i < nslot / 2; i += kFinBlock) gw[i] = ltag[i];
    v2i64* gs = reinterpret_cast<v2i64*>(table_slots(h, cap_max)) + ((size_t)d << log2g) * kBucket;
    for (int i = tid; i < nslot; i += kFinBlock) gs[i] = lslot[i];
  };
  if (!multi) {
    each_row([&](const v2i64& kv) {
      const uint64_t hh = mulhash(kv.x);
      add_bloom(hh);
      insert(kv, hh);
    });
    __syncthreads();
    write_domain(j);
  } else {
    const int nsub = 1 << sub_log2;
    auto sub_of = [&](uint64_t hh) {
      return (int)((bucket_of(hh, skip, l - kLog2Bucket) >> log2g) & (uint64_t)(nsub - 1));
    };
    // count the rows of each domain; each must keep an eighth of its slots free
    each_row([&](const v2i64& kv) {
      const uint64_t hh = mulhash(kv.x);
      add_bloom(hh);
      atomicAdd(&sub_cnt[sub_of(hh)], 1u);
    });
    __syncthreads();
    bool ok = true;
    for (int d = 0; d < nsub; d++) ok = ok && sub_cnt[d] <= (uint32_t)(kMaxRegionSlots - kMaxRegionSlots / 8);
    if (!ok) {
      if (tid == 0) atomicOr(&h->ovf, 1);
      return;
    }
    if (tid == 0) {
      sub_off[0] = 0;
      for (int d = 0; d < nsub; d++) sub_off[d + 1] = sub_off[d] + sub_cnt[d];
    }
    __syncthreads();
    // stage the rows grouped by domain at the front of the region's own slot
    // area: domain d's rows end below d * kMaxRegionSlots (each domain holds
    // fewer), so filling the domains from the last one down never overwrites
    // rows not yet read
    v2i64* stage = reinterpret_cast<v2i64*>(table_slots(h, cap_max)) + ((size_t)j << (l - kLog2Bins));
    each_row([&](const v2i64& kv) {
      const int d = sub_of(mulhash(kv.x));
      stage[sub_off[d] + atomicAdd(&sub_fill[d], 1u)] = kv;
    });
    __syncthreads();
    for (int d = nsub - 1; d >= 0; d--) {
      ltag[tid] = 0u;
      __syncthreads();
      for (uint32_t r = sub_off[d] + tid; r < sub_off[d + 1]; r += kFinBlock) {
        const v2i64 kv = stage[r];
        insert(kv, mulhash(kv.x));
      }
      __syncthreads();
      write_domain(((int64_t)j << sub_log2) + d);
      __syncthreads();
    }
  }
  if (stuck) latch_error(&h->err, TQ_EFULL);
  for (int i = tid; i < nbw; i += kFinBlock) scratch_bloom(h, cap_max)[(size_t)j * nbw + i] = lbloom[i];
}

constexpr int kFallbackBlocks = 16;  // two per XCD, for tables that cannot leave the regions' range

template <int NC>
__global__ __launch_bounds__(kBlock) void k_build_fallback(RowPlan P, const int64_t* keys, DCol payload, int64_t n,
                                                          TableHeader* h, int64_t cap_max, const uint8_t* key_valid) {
  if (h->magic != kTableMagic || !h->ovf) return;
  const int l = h->log2cap, skip = h->skip;
  const uint32_t flags = h->flags;
  const bool nulls = P.null_cols != 0 || key_valid != nullptr;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->regions = 0;
    h->alt = 1;
    h->log2g = l - kLog2Bucket;
    h->bloom_log2w = 0;
  }
  uint32_t* words = scratch_alt_tags(h, cap_max);
  v2i64* slots = reinterpret_cast<v2i64*>(scratch_rows(h, cap_max));
  const DCol kc = {keys, 8};
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kRows;
  for (int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRows; r0 < n; r0 += step) {
    const bool fullrow = r0 + kRows <= n;
    int64_t v[NC][kRows], k[kRows], pay[kRows];
    bool pend[kRows];
    load_rows<NC>(P, r0, fullrow, n, v);
    load4(kc, r0, fullrow, n, k);
    load4(payload, r0, fullrow, n, pay);
#pragma unroll
    for (int i = 0; i < kRows; i++) {
      pend[i] = (r0 + i < n) && build_row_ok<NC>(P, v, i, r0 + i, key_valid, nulls) &&
                in_partition(mulhash(k[i]), skip, flags);
      if (pend[i]) pay[i] = stored_payload(payload, r0 + i, pay[i]);
    }
    table_insert<kRows>(words, slots, l, skip, pend, k, pay);
  }
}

// ------------------------------------------------------------------ probe

// With NULLs (a validity bitmap on the probe key, on a plan column, or a
// nullable state): a NULL probe key matches nothing, a predicate over NULL
// drops the row, a match whose stored payload is INT64_MIN (a NULL build
// payload) goes to the NULL group, and a sum reading a NULL value skips it.
template <int MODE, int NC, int NE>
__global__ __launch_bounds__(kAggBlock, kAggBlocksPerCU) void k_probe_agg(const TableHeader* h, const int64_t* pkeys, int64_t n, RowPlan P,
                                                         AggTarget T, const uint8_t* key_valid) {
  extern __shared__ __align__(16) char smem[];
  if (h->magic != kTableMagic || h->err) return;  // a failed build inserted nothing: no row can match
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
  const bool nulls = P.null_cols != 0 || key_valid != nullptr;
  for (; r0 < n; r0 += step) {
    int64_t k[kPR], e[kPR][NE];
    bool ok[kPR];
    uint32_t epresent[kPR];  // bit j: sum j reads no NULL value in the row
#pragma unroll
    for (int i = 0; i < kPR; i++) {
      epresent[i] = ~0u;
      if (!nulls) {
        ok[i] = (r0 + i < n) && eval_preds<NC>(P, vn, i);
      } else {
        const uint32_t present = r0 + i < n ? row_present<NC>(P, r0 + i) : 0u;
        ok[i] = (r0 + i < n) && (!key_valid || bit_at(key_valid, r0 + i)) &&
                eval_preds_present<NC>(P, vn, i, present);
#pragma unroll
        for (int j = 0; j < NE; j++) {
          const uint32_t ec = j < P.ne ? expr_cols(P.expr[j]) : 0u;
          if ((present & ec) != ec) epresent[i] &= ~(1u << j);
        }
      }
#pragma unroll
      for (int j = 0; j < NE; j++) e[i][j] = j < P.ne ? eval_expr<NC>(P.expr[j], vn, i) : 0;
      k[i] = kn[i];
    }
    const int64_t r1 = r0 + step;
    pr.walk(
        ok, k,
        [&](const bool (&hit)[kPR], const int64_t (&pay)[kPR]) {
#pragma unroll
          for (int i = 0; i < kPR; i++) {
            if (!hit[i]) continue;
            if (T.nullable) {
              // INT64_MIN: a NULL build payload (the NULL group); a present one outside the domain: an error
              const int64_t g = pay[i] == INT64_MIN ? T.udomain
                                                    : ((uint64_t)pay[i] < (uint64_t)T.udomain ? pay[i] : -1);
              agg.add_nullable(T, g, e[i], epresent[i], P.ne);
            } else {
              agg.add(T, pay[i], e[i], P.ne);
            }
          }
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

// ---------------------------------------------------------------------------
// Pipelined probe with the fused group-by (int64 columns, up to two sums).
//
// Each lane takes two consecutive rows per tile (one 16-byte load per column);
// tiles are strided over the grid. Four tiles of a lane are in flight at
// once, one per stage: in iteration j the candidate slots of tile j are
// consumed, the tags of tile j+1 turn into slot loads, the columns of tile j+2
// into tag loads, and the columns of tile j+3 are requested. Each load is
// issued one iteration before its data is used, and the loads of an
// iteration are issued in the order they are consumed, so every wait covers
// only the oldest loads. Every load is issued unconditionally: a row with
// nothing to read loads a fixed valid address instead (one line shared by the
// wave), so the count of loads in flight is the same on every path. The row of
// a partial last tile (at most one) is walked by one lane at the end.
//
// A row is finished from its home bucket alone when the bucket decides it: no
// tag match and a free slot (a miss), exactly one candidate and a free slot
// (hit or miss), or a hit on unique build keys. Any other row (a full home
// bucket, further candidates) goes to a queue in LDS private to its wave. A
// queued row starts again from its home bucket and nothing of it was
// aggregated before, so every match is counted exactly once. The queue is
// walked (64 rows at a time, each to the end of its chain) only outside the
// pipelined loop: at its end, or when the queue could not take another
// iteration's rows, in which case the loop stops before finishing anything of
// the tiles in flight, the queue is walked, and the loop starts again at the
// first unfinished tile. (A walk inside the loop would wait for every load in
// flight, and the compiler then also waits for all of them on the loop's own
// path, as a register the walk loads into is one the loop reuses.)
//
// With BLOOM, the workgroup holds the build's Bloom filter in LDS (one
// workgroup per CU, for its 128 KiB) and a row the filter rejects is not live:
// its tag load goes to the shared dummy line, so a probe key the build does
// not hold costs no table traffic. A table without a filter (a fallback
// build) passes every row.
#ifndef TQ_PIPE_BLOCKS_PER_CU
#define TQ_PIPE_BLOCKS_PER_CU 2
#endif
constexpr int kPipeBlocksPerCU = TQ_PIPE_BLOCKS_PER_CU;
constexpr int kPipeRows = 2;
constexpr int kPipeQ = 320;  // queue entries per wave (row offsets from the wave's first row, 4 bytes)
// the loop goes on only while the queue can take the two tiles an iteration finishes
constexpr int kPipeQLimit = kPipeQ - 2 * kWave * kPipeRows;
static_assert(kPipeQLimit >= 0, "queue");
// rows per launch of the pipelined probe: queued rows are kept as 32-bit offsets
constexpr int64_t kPipeMaxRows = (int64_t)1 << 31;
constexpr int kBloomPipeBlock = 1024;  // one workgroup per CU beside the filter: 16 waves
constexpr size_t kMaxPipeLds = 64 * 1024;  // dynamic LDS of a launch without a per-kernel attribute
constexpr size_t kCuLds = 160 * 1024;
constexpr size_t kMaxBloomPipeLds = kCuLds - (size_t)kBloomWordsMax * 4;  // dynamic LDS beside the filter

template <int NE>
struct PipeRows {
  static constexpr int R = kPipeRows;
  int64_t k[R], e[R][NE], b[R];
  int64_t row;  // the tile's first row
  uint32_t tg[R];
  bool live[R];
};

// A sum as a product of up to three (column + constant) factors, negated when
// `neg` is set: the form of every expression whose coefficients are 1, -1 or 0
// (add - x = -(x + (-add)) mod 2^64; a constant factor has a zero column mask,
// which picks 0 from at most two columns). It needs no 64-bit multiply by a
// coefficient (three quarter-rate instructions each on this GPU).
struct UnitSum {
  int32_t nf;
  int32_t neg;
  uint32_t mask[3];
  int64_t add[3];
};
struct UnitPlan {
  UnitSum s[2];
};

// The unit form of the plan's sums; false if some coefficient is not 1, -1 or 0.
static bool unit_plan(const RowPlan& P, UnitPlan* U) {
  *U = UnitPlan{};
  for (int j = 0; j < P.ne; j++) {
    if (j >= 2) return false;
    UnitSum& S = U->s[j];
    S.nf = P.expr[j].nf;
    for (int f = 0; f < S.nf; f++) {
      const DFactor& F = P.expr[j].f[f];
      if (F.sign == 0) {
        S.mask[f] = 0u;
        S.add[f] = F.add;
      } else if (F.sign == 1 || F.sign == -1) {
        S.mask[f] = F.mask;
        S.add[f] = F.sign == 1 ? F.add : (int64_t)(0ull - (uint64_t)F.add);
        S.neg ^= F.sign == -1;
      } else {
        return false;
      }
    }
  }
  return true;
}

template <int NC, int R>
__device__ __forceinline__ int64_t eval_unit(const UnitSum& S, const int64_t (&v)[NC][R], int i) {
  static_assert(NC <= 2, "a zero mask must pick 0");
  uint64_t acc = (uint64_t)pick<NC, R>(v, i, S.mask[0]) + (uint64_t)S.add[0];
#pragma unroll
  for (int f = 1; f < 3; f++)
    if (f < S.nf) acc *= (uint64_t)pick<NC, R>(v, i, S.mask[f]) + (uint64_t)S.add[f];
  return (int64_t)(S.neg ? 0ull - acc : acc);
}

// FAST: the common plan (group-by partials dense in LDS, at most two columns,
// no probe-side predicate, sums of unit coefficients; U holds them): no
// predicate loop, sums without multiplies by a coefficient, and the LDS adds
// of a match in one branch with no call into the generic group-by code, so
// that the few values they need stay in scalar registers.
template <int MODE, int NC, int NE, bool BLOOM, bool FAST>
__global__ __launch_bounds__(BLOOM ? kBloomPipeBlock : kAggBlock, BLOOM ? 1 : kPipeBlocksPerCU) void k_probe_pipe(const TableHeader* h,
                                                                                        const int64_t* pkeys, int64_t n,
                                                                                        RowPlan P, AggTarget T,
                                                                                        UnitPlan U, int agg_lds) {
  static_assert(!FAST || (MODE == kDense && NC <= 2), "fast plan");
  constexpr int R = kPipeRows;
  __shared__ uint32_t bloom[BLOOM ? kBloomWordsMax : 1];
  extern __shared__ __align__(16) char smem[];
  if (h->magic != kTableMagic || h->err) return;  // a failed build inserted nothing: no row can match
  if (!state_matches(T)) return;
  // (a filter larger than the LDS copy, in device memory only, is not used here)
  const int log2w = BLOOM && h->bloom_log2w <= kLog2BloomWordsMax ? h->bloom_log2w : 0;
  const int nbw = log2w ? 1 << log2w : 0;
  if (BLOOM) {
    // every load of the copy first, then every LDS store: one round trip to
    // memory instead of one per 16 bytes a thread copies
    constexpr int kU = kBloomWordsMax / 4 / kBloomPipeBlock;
    static_assert(kU * 4 * kBloomPipeBlock == kBloomWordsMax, "filter copy");
    const v4i32* gb = reinterpret_cast<const v4i32*>(scratch_bloom(const_cast<TableHeader*>(h), h->cap_max));
    v4i32 t[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int i = (int)threadIdx.x + u * kBloomPipeBlock;
      if (i < nbw / 4) t[u] = gb[i];
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int i = (int)threadIdx.x + u * kBloomPipeBlock;
      if (i < nbw / 4) reinterpret_cast<v4i32*>(bloom)[i] = t[u];
    }
  }
  LdsAgg<MODE> agg;
  agg.defer = true;
  agg.init(T, smem);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t* qrow = reinterpret_cast<uint32_t*>(smem + agg_lds) + (int64_t)wave * kPipeQ;  // queued rows
  // (the barrier after which the filter, the partials and the queues may be
  // used comes after the first tiles' column loads, which it overlaps)
  Probe pr;
  pr.setup(h);
  const int64_t n_main = n & ~(int64_t)(R - 1);  // rows in full tiles
  const v2i64* kcol = reinterpret_cast<const v2i64*>(pkeys);
  const v2i64* ccol[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) ccol[c] = c < P.ncol ? static_cast<const v2i64*>(P.col[c].p) : kcol;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * R;
  const int64_t wbase = ((int64_t)blockIdx.x * blockDim.x + wave * kWave) * R;  // the wave's first row
  int qn = 0;  // queued rows (the same in every lane); the queue is only appended to inside the loop
  const int ne = P.ne;
  const uint64_t udomain = (uint64_t)T.domain;
  const uint32_t gstride = (uint32_t)T.stride;  // entries per group: COUNT and the sums
  bool bad = false;  // FAST: a group key outside the domain was met

  // Walks every queued row to the end of its chain, 64 at a time, one per lane
  // (their key and columns are read again: queued rows are rare), and empties
  // the queue.
  auto drain_all = [&] {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int q0 = 0; q0 < qn; q0 += kWave) {
      bool ok1[1] = {q0 + lane < qn};
      int64_t k1[1] = {0}, e1[NE];
#pragma unroll
      for (int j = 0; j < NE; j++) e1[j] = 0;
      if (ok1[0]) {
        const int64_t row = wbase + qrow[q0 + lane];
        int64_t v1[NC][1];
#pragma unroll
        for (int c = 0; c < NC; c++) v1[c][0] = c < P.ncol ? reinterpret_cast<const int64_t*>(ccol[c])[row] : 0;
        k1[0] = pkeys[row];
#pragma unroll
        for (int j = 0; j < NE; j++) e1[j] = j < P.ne ? eval_expr<NC>(P.expr[j], v1, 0) : 0;
      }
      pr.walk(ok1, k1, [&](const bool (&hit)[1], const int64_t (&pay)[1]) {
        if (hit[0]) agg.add(T, pay[0], e1, P.ne);
      });
    }
    qn = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };

  bool first = true;  // the one workgroup barrier comes in the first prologue (or below)
  int64_t pos = wbase;  // this wave's first tile not yet finished
  while (pos < n_main) {
    int64_t r = pos + lane * R;
    v2i64 cva[NC], cka, cvb[NC], ckb;  // columns of two tiles ahead (alternating sets)
    v4i32 tw[R];            // tags of the tile 1 ahead
    v2i64 kv[R];            // candidate slots of the current tile
    PipeRows<NE> ra, rb;    // row state of two consecutive tiles (alternating sets, never copied)
    uint32_t sm[R];         // candidate masks of the home buckets (slot loads in flight)
    bool sempty[R];         // the home bucket has a free slot

    auto load_cols = [&](v2i64 (&cv)[NC], v2i64& ck, int64_t rt) {  // a tile past the last reads tile 0
      const int64_t q = (rt < n_main ? rt : 0) / R;
      ck = ntload(kcol + q);
#pragma unroll
      for (int c = 0; c < NC; c++) cv[c] = ntload(ccol[c] + q);
    };
    auto cols_to_tags = [&](const v2i64 (&cv)[NC], const v2i64& ck, int64_t rt, PipeRows<NE>& t) {  // -> t; tag loads
      int64_t v[NC][R];
#pragma unroll
      for (int c = 0; c < NC; c++) {
        v[c][0] = cv[c].x;
        v[c][1] = cv[c].y;
      }
      const int64_t kk[R] = {ck.x, ck.y};
      t.row = rt;
#pragma unroll
      for (int i = 0; i < R; i++) {
        if constexpr (FAST) {
          t.live[i] = rt < n_main;
#pragma unroll
          for (int j = 0; j < NE; j++) t.e[i][j] = j < ne ? eval_unit<NC>(U.s[j], v, i) : 0;
        } else {
          t.live[i] = (rt < n_main) && eval_preds<NC>(P, v, i);
#pragma unroll
          for (int j = 0; j < NE; j++) t.e[i][j] = j < ne ? eval_expr<NC>(P.expr[j], v, i) : 0;
        }
        t.k[i] = kk[i];
        const uint64_t hh = mulhash(kk[i]);
        t.live[i] = t.live[i] && pr.selected(hh);
        t.b[i] = (int64_t)bucket_of(hh, pr.skip, pr.log2b);
        t.tg[i] = hash_tag(hh);
        if (BLOOM && nbw) {  // a key the filter rejects is not in the build
          const uint32_t m = bloom_bits(hh);
          t.live[i] = t.live[i] && (bloom[bloom_word(hh, pr.skip, log2w)] & m) == m;
        }
      }
#pragma unroll
      for (int i = 0; i < R; i++) tw[i] = pr.groups[t.live[i] ? t.b[i] : 0];
    };
    auto tags_to_slots = [&](const PipeRows<NE>& t) {  // tw -> candidate masks; slot loads
#pragma unroll
      for (int i = 0; i < R; i++) {
        sm[i] = t.live[i] ? tag_match(tw[i], t.tg[i]) : 0u;
        sempty[i] = t.live[i] ? has_empty(tw[i]) : true;
      }
#pragma unroll
      for (int i = 0; i < R; i++) kv[i] = pr.slots[sm[i] ? t.b[i] * kBucket + __builtin_ctz(sm[i]) : 0];
    };
    // (a) finish a tile from its slots (before any register they live in is
    // reloaded); rows the home bucket does not decide go to the queue
    auto finish = [&](const PipeRows<NE>& t) {
#pragma unroll
      for (int i = 0; i < R; i++) {
        const bool cand = sm[i] != 0u;
        const bool hit = cand && kv[i].x == t.k[i];
        const uint32_t rest = sm[i] & (sm[i] - 1u);
        const bool done =
            !t.live[i] || (sm[i] == 0u && sempty[i]) || (hit && pr.unique) || (rest == 0u && sempty[i]);
        if constexpr (FAST) {
          const bool addit = done && hit;
          const uint64_t key = (uint64_t)kv[i].y;
          const bool in = key < udomain;
          bad = bad || (addit && !in);  // latched after the loop
          if (addit && in) {  // key < domain <= 4096 (dense partials): a 24-bit multiply
            unsigned long long* d = reinterpret_cast<unsigned long long*>(agg.vals) + __umul24((uint32_t)key, gstride);
            atomicAdd(d, 1ull);
#pragma unroll
            for (int j = 0; j < NE; j++)
              if (j < ne) atomicAdd(d + 1 + j, (unsigned long long)t.e[i][j]);
          }
        } else {
          if (done && hit) agg.add(T, kv[i].y, t.e[i], ne);
        }
        const bool slow = !done;
        const uint64_t bal = __ballot(slow);
        if (bal) {
          if (slow) {
            const int rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            qrow[qn + rank] = (uint32_t)(t.row + i - wbase);
          }
          qn += __popcll(bal);
        }
      }
    };

    // prologue: tile 0 to its slot loads (row state ra), tile 1 to its tag
    // loads (rb), tiles 2 and 3's columns requested
    load_cols(cva, cka, r);
    load_cols(cvb, ckb, r + stride);
    asm volatile("" ::: "memory");
    if (first) __syncthreads();
    first = false;
    cols_to_tags(cva, cka, r, ra);
    asm volatile("" ::: "memory");
    tags_to_slots(ra);
    asm volatile("" ::: "memory");
    cols_to_tags(cvb, ckb, r + stride, rb);
    asm volatile("" ::: "memory");
    load_cols(cva, cka, r + 2 * stride);
    asm volatile("" ::: "memory");
    load_cols(cvb, ckb, r + 3 * stride);
    asm volatile("" ::: "memory");
    // Two tiles per pass, one per column set and row-state set, so that each
    // set's loads have two tiles' time to arrive. Per tile: (a) finish it; (b)
    // the next tile's tags -> slot loads; (c) the tile two ahead: columns ->
    // tag loads, into the row state just finished; (d) request the columns
    // four ahead. The empty asm statements keep each stage's loads where they
    // are: the compiler would otherwise merge them with later ones, after the
    // loads they must precede. A second tile past the wave's last reads tile 0
    // and is not live. The pass stops early, finishing nothing of the tiles in
    // flight, when the queue could not take its rows.
    int64_t w0 = pos;
    for (; w0 < n_main; w0 += 2 * stride, r += 2 * stride) {
      if (qn > kPipeQLimit) break;
      finish(ra);
      tags_to_slots(rb);
      asm volatile("" ::: "memory");
      cols_to_tags(cva, cka, r + 2 * stride, ra);
      asm volatile("" ::: "memory");
      load_cols(cva, cka, r + 4 * stride);
      asm volatile("" ::: "memory");
      finish(rb);
      tags_to_slots(ra);
      asm volatile("" ::: "memory");
      cols_to_tags(cvb, ckb, r + 3 * stride, rb);
      asm volatile("" ::: "memory");
      load_cols(cvb, ckb, r + 5 * stride);
      asm volatile("" ::: "memory");
    }
    pos = w0;  // every tile before w0 is finished (its queued rows are in the queue)
    if (qn > 0) drain_all();
  }
  if (first) __syncthreads();  // a wave with no full tile still takes part in the barrier
  if (qn > 0) drain_all();
  if (n_main < n && blockIdx.x == 0 && threadIdx.x == 0) {
    // the row of the partial last tile
    const int64_t rt = n_main;
    int64_t v[NC][1];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c][0] = c < P.ncol ? static_cast<const int64_t*>(P.col[c].p)[rt] : 0;
    bool ok1[1] = {eval_preds<NC>(P, v, 0)};
    int64_t k1[1] = {pkeys[rt]}, e1[NE];
#pragma unroll
    for (int j = 0; j < NE; j++) e1[j] = j < P.ne ? eval_expr<NC>(P.expr[j], v, 0) : 0;
    pr.walk(ok1, k1, [&](const bool (&hit)[1], const int64_t (&pay)[1]) {
      if (hit[0]) agg.add(T, pay[0], e1, P.ne);
    });
  }
  agg.bad = agg.bad || bad;
  agg.flush(T);
}

// The fast aggregating probe behind the Bloom filter with the rows that pass
// the filter compacted across the wave before the table stages. Most probe
// rows have no partner and the filter drops most of those; the tag, slot and
// aggregation stages then run on 64-row tiles of the survivors instead of on
// every row slot. Stage 1, per tile of 2 rows per lane (columns requested
// two tiles ahead): hash and filter test (the filter in LDS, or in device
// memory when it is larger than the LDS copy: tables past 2^19 slots); the
// survivors move to the wave's compaction buffer (three 64-row register
// tiles, B0, B1, B2) with one ds_permute per 32-bit word: survivors to the
// buffer's next free lanes, the rest to the remaining lanes, so the lane map
// is a permutation. Stage 2, once per two tiles (and before a tile when the
// buffer might not take its rows): the buffer's first tile (full, or what
// there is) goes through a three-deep pipeline: its tag loads are issued;
// the tile before it turns its tags into slot loads; the one before that is
// finished (aggregated, or queued for the chain walk).
constexpr int kCmpSets = 2;  // column tiles in flight per wave (even)
constexpr int kCmpQLimit = kPipeQ - kWave;  // a finish queues at most 64 rows

// A compacted row: its key, its sum's value (evaluated before the row is
// compacted: fewer words to move and to hold), its offset from the wave's
// first row.
struct CRow {
  int64_t k, e;
  uint32_t r;
};
__device__ __forceinline__ CRow crow_select(bool take, const CRow& a, const CRow& b) {
  return CRow{take ? a.k : b.k, take ? a.e : b.e, take ? a.r : b.r};
}

template <int NC, int NE>
__global__ __launch_bounds__(kBloomPipeBlock, 1) void k_probe_compact(const TableHeader* h, const int64_t* pkeys,
                                                                      int64_t n, RowPlan P, AggTarget T, UnitPlan U,
                                                                      int agg_lds) {
  static_assert(NC <= 2 && NE == 1, "fast plan with one sum");
  constexpr int R = kPipeRows;
  __shared__ uint32_t bloom[kBloomWordsMax];
  extern __shared__ __align__(16) char smem[];
  if (h->magic != kTableMagic || h->err) return;  // a failed build inserted nothing: no row can match
  if (!state_matches(T)) return;
  const int log2w = h->bloom_log2w;
  const int nbw = log2w ? 1 << log2w : 0;
  // a filter past the LDS copy's size is read from device memory (the same
  // choice in every lane)
  const bool gfilter = nbw > kBloomWordsMax;
  const uint32_t* gbloom = scratch_bloom(const_cast<TableHeader*>(h), h->cap_max);
  if (!gfilter) {
    constexpr int kU = kBloomWordsMax / 4 / kBloomPipeBlock;
    const v4i32* gb = reinterpret_cast<const v4i32*>(gbloom);
    v4i32 t[kU];
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int i = (int)threadIdx.x + u * kBloomPipeBlock;
      if (i < nbw / 4) t[u] = gb[i];
    }
#pragma unroll
    for (int u = 0; u < kU; u++) {
      const int i = (int)threadIdx.x + u * kBloomPipeBlock;
      if (i < nbw / 4) reinterpret_cast<v4i32*>(bloom)[i] = t[u];
    }
  }
  LdsAgg<kDense> agg;
  agg.defer = true;
  agg.init(T, smem);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t* qrow = reinterpret_cast<uint32_t*>(smem + agg_lds) + (int64_t)wave * kPipeQ;  // queued rows
  Probe pr;
  pr.setup(h);
  const int64_t n_main = n & ~(int64_t)(R - 1);  // rows in full tiles
  const v2i64* kcol = reinterpret_cast<const v2i64*>(pkeys);
  const v2i64* ccol[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) ccol[c] = c < P.ncol ? static_cast<const v2i64*>(P.col[c].p) : kcol;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * R;
  const int64_t wbase = ((int64_t)blockIdx.x * blockDim.x + wave * kWave) * R;  // the wave's first row
  int qn = 0;
  const int ne = P.ne;
  const uint64_t udomain = (uint64_t)T.domain;
  const uint32_t gstride = (uint32_t)T.stride;
  bool bad = false;

  auto drain_all = [&] {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int q0 = 0; q0 < qn; q0 += kWave) {
      bool ok1[1] = {q0 + lane < qn};
      int64_t k1[1] = {0}, e1[NE];
#pragma unroll
      for (int j = 0; j < NE; j++) e1[j] = 0;
      if (ok1[0]) {
        const int64_t row = wbase + qrow[q0 + lane];
        int64_t v1[NC][1];
#pragma unroll
        for (int c = 0; c < NC; c++) v1[c][0] = c < P.ncol ? reinterpret_cast<const int64_t*>(ccol[c])[row] : 0;
        k1[0] = pkeys[row];
#pragma unroll
        for (int j = 0; j < NE; j++) e1[j] = j < P.ne ? eval_expr<NC>(P.expr[j], v1, 0) : 0;
      }
      pr.walk(ok1, k1, [&](const bool (&hit)[1], const int64_t (&pay)[1]) {
        if (hit[0]) agg.add(T, pay[0], e1, P.ne);
      });
    }
    qn = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };

  // the compaction buffer: B0, B1, B2, `fill` rows (the same in every lane)
  CRow B0{0, 0, 0u}, B1 = B0, B2 = B0;
  int fill = 0;
  // stage 2: Y has its tag loads in flight, X its slot loads
  CRow Y = B0, X = B0;
  uint32_t ytg = 0, yb = 0, xsm = 0;
  bool yv = false, xv = false, xse = true;
  v4i32 ytw = v4i32{0, 0, 0, 0};
  v2i64 xkv = v2i64{0, 0};

  // One step of stage 2, with Z (valid lanes: zv) entering it.
  auto advance = [&](bool zv, const CRow Z) {
    {  // finish X
      const bool hit = xsm != 0u && xkv.x == X.k;
      const uint32_t rest = xsm & (xsm - 1u);
      const bool done = !xv || (xsm == 0u && xse) || (hit && pr.unique) || (rest == 0u && xse);
      const bool addit = done && hit;
      const uint64_t key = (uint64_t)xkv.y;
      const bool in = key < udomain;
      bad = bad || (addit && !in);  // latched after the loop
      if (addit && in) {  // key < domain <= 4096 (dense partials): a 24-bit multiply
        unsigned long long* d = reinterpret_cast<unsigned long long*>(agg.vals) + __umul24((uint32_t)key, gstride);
        atomicAdd(d, 1ull);
        if (ne > 0) atomicAdd(d + 1, (unsigned long long)X.e);
      }
      const bool slow = !done;
      const uint64_t bal = __ballot(slow);
      if (bal) {
        if (slow) {
          const int rank =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          qrow[qn + rank] = X.r;
        }
        qn += __popcll(bal);
      }
    }
    {  // Y -> X: tags to slot loads
      X = Y;
      xv = yv;
      xsm = yv ? tag_match(ytw, ytg) : 0u;
      xse = yv ? has_empty(ytw) : true;
      xkv = pr.slots[xsm ? (int64_t)yb * kBucket + __builtin_ctz(xsm) : 0];
    }
    asm volatile("" ::: "memory");
    {  // Z -> Y: tag loads
      const uint64_t hh = mulhash(Z.k);
      Y = Z;
      yv = zv;
      yb = (uint32_t)bucket_of(hh, pr.skip, pr.log2b);
      ytg = hash_tag(hh);
      ytw = pr.groups[zv ? yb : 0u];
    }
    asm volatile("" ::: "memory");
    if (qn > kCmpQLimit) drain_all();
  };
  // B0 (its first min(fill, 64) rows) into stage 2; the others move up
  auto emit = [&] {
    const int cnt = fill < kWave ? fill : kWave;
    advance(lane < cnt, B0);
    B0 = B1;
    B1 = B2;
    fill = fill > kWave ? fill - kWave : 0;
  };
  // appends the lanes' rows with `live` set to the buffer (fill <= 128)
  auto push = [&](bool live, const CRow& row) {
    const uint64_t m = __ballot(live);
    if (m == 0) return;
    const int cnt = __popcll(m);
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const int addr = ((fill + (live ? rank : cnt + lane - rank)) & (kWave - 1)) * 4;
    auto perm32 = [&](uint32_t x) { return (uint32_t)__builtin_amdgcn_ds_permute(addr, (int)x); };
    auto perm = [&](int64_t x) {
      const uint32_t lo = perm32((uint32_t)x), hi = perm32((uint32_t)((uint64_t)x >> 32));
      return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    const CRow rv{perm(row.k), perm(row.e), perm32(row.r)};
    // the tile holding position `fill` takes the new rows from lane fill % 64
    // on; rows past its end land in the lanes below and start the next tile
    // (selects, not branches: stores under a branch would be merged into
    // indexed ones, and the buffer would live in scratch memory)
    const bool take = lane >= (fill & (kWave - 1));
    const int t = fill >> 6;  // 0, 1, or 2 (fill == 128)
    B2 = crow_select(t == 1 || (t == 2 && take), rv, B2);
    B1 = crow_select(t == 0 || (t == 1 && take), rv, B1);
    B0 = crow_select(t == 0 && take, rv, B0);
    fill += cnt;
  };
  // stage 1 of one tile (rows rt, rt + 1 of each lane)
  auto stage1 = [&](const v2i64 (&cv)[NC], const v2i64& ck, int64_t rt) {
    const int64_t kk[R] = {ck.x, ck.y};
    int64_t v[NC][R];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      v[c][0] = cv[c].x;
      v[c][1] = cv[c].y;
    }
#pragma unroll
    for (int i = 0; i < R; i++) {
      const uint64_t hh = mulhash(kk[i]);
      bool live = rt < n_main && pr.selected(hh);
      if (nbw) {  // a key the filter rejects is not in the build
        const uint32_t wd = bloom_word(hh, pr.skip, log2w);
        // (each branch tests its own load: a use after the branches would
        // wait for the loads of both kinds)
        if (gfilter) {
          const uint32_t m = bloom_bits(hh, log2w);
          live = live && (gbloom[rt < n_main ? wd : 0u] & m) == m;
        } else {
          const uint32_t m = bloom_bits(hh);  // (log2w <= kLog2BloomWordsMax)
          live = live && (bloom[wd] & m) == m;
        }
      }
      const CRow row{kk[i], ne > 0 ? eval_unit<NC>(U.s[0], v, i) : 0, (uint32_t)(rt + i - wbase)};
      push(live, row);
    }
  };
  auto load_cols = [&](v2i64 (&cv)[NC], v2i64& ck, int64_t rt) {  // a tile past the last reads tile 0
    const int64_t q = (rt < n_main ? rt : 0) / R;
    ck = ntload(kcol + q);
#pragma unroll
    for (int c = 0; c < NC; c++) cv[c] = ntload(ccol[c] + q);
  };

  v2i64 cv[kCmpSets][NC], ck[kCmpSets];
  int64_t r = wbase + lane * R;
  if (n_main > 0) {  // (with no full tile there is no tile 0 to read in its place)
#pragma unroll
    for (int s = 0; s < kCmpSets; s++) load_cols(cv[s], ck[s], r + s * stride);
  }
  asm volatile("" ::: "memory");
  __syncthreads();  // the filter, the partials and the queues are ready
  for (int64_t t0 = wbase; t0 < n_main; t0 += kCmpSets * stride, r += kCmpSets * stride) {
#pragma unroll
    for (int s = 0; s < kCmpSets; s++) {
      while (fill > kWave) emit();  // (rare) so that the buffer takes this tile's 128 rows
      stage1(cv[s], ck[s], r + s * stride);
      asm volatile("" ::: "memory");
      load_cols(cv[s], ck[s], r + (s + kCmpSets) * stride);
      asm volatile("" ::: "memory");
      if (s & 1) emit();
    }
  }
  while (fill > 0) emit();
  advance(false, CRow{0, 0, 0u});
  advance(false, CRow{0, 0, 0u});
  if (qn > 0) drain_all();
  if (n_main < n && blockIdx.x == 0 && threadIdx.x == 0) {
    // the row of the partial last tile
    const int64_t rt = n_main;
    int64_t v[NC][1];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c][0] = c < P.ncol ? static_cast<const int64_t*>(P.col[c].p)[rt] : 0;
    bool ok1[1] = {eval_preds<NC>(P, v, 0)};
    int64_t k1[1] = {pkeys[rt]}, e1[NE];
#pragma unroll
    for (int j = 0; j < NE; j++) e1[j] = j < P.ne ? eval_expr<NC>(P.expr[j], v, 0) : 0;
    pr.walk(ok1, k1, [&](const bool (&hit)[1], const int64_t (&pay)[1]) {
      if (hit[0]) agg.add(T, pay[0], e1, P.ne);
    });
  }
  agg.bad = agg.bad || bad;
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
  // a failed build inserted nothing: its rows count no match (and its tags are not cleared)
  const int64_t lo = (int64_t)blockIdx.x * per, hi = h->err ? lo : min(n, lo + per);
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
  if (h->magic != kTableMagic || h->err) return;  // a failed build: every block counted no match
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

tq_status tq_join_table_rows(const void* d_table, int64_t* rows, hipStream_t stream) {
  if (!d_table || !rows) return fail(TQ_EINVAL, "NULL argument");
  TableHeader hdr;
  TQ_HIP(hipMemcpyAsync(&hdr, d_table, sizeof hdr, hipMemcpyDeviceToHost, stream));
  TQ_HIP(hipStreamSynchronize(stream));
  if (hdr.magic != kTableMagic) return fail(TQ_EINVAL, "not a join table");
  *rows = hdr.n;
  return TQ_OK;
}

}  // extern "C"

static tq_status join_build(void* d_table, size_t bytes, const int64_t* d_keys, const uint8_t* key_valid,
                            tq_col payload, int64_t n, const tq_col* filt, int32_t nfilt, const tq_pred* p, int32_t np,
                            double load_factor, int32_t skip, uint32_t flags, bool nullable, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (!(load_factor > 0.0 && load_factor <= 0.9)) return fail(TQ_EINVAL, "load factor %g outside (0, 0.9]", load_factor);
  if (skip < 0 || skip > 32) return fail(TQ_EINVAL, "skip %d outside [0, 32]", skip);
  if (flags & ~(TQ_UNIQUE_KEYS | TQ_SELECT_PARTITION | TQ_PARTITION(0xffffu)))
    return fail(TQ_EINVAL, "unknown flags 0x%x", flags);
  if (flags & TQ_SELECT_PARTITION) {
    if (skip < 1 || skip > 16) return fail(TQ_EINVAL, "a partition build needs 1 <= skip <= 16 (got %d)", skip);
    if ((flags >> 16) >= (1u << skip)) return fail(TQ_EINVAL, "partition %u outside [0, 2^%d)", flags >> 16, skip);
  } else if (flags >> 16) {
    return fail(TQ_EINVAL, "a partition id without TQ_SELECT_PARTITION");
  }
  if (n < 0) return fail(TQ_EINVAL, "n < 0");
  if (n > 0 && (!d_keys || !payload.data)) return fail(TQ_EINVAL, "NULL keys or payload");
  if (((uintptr_t)d_keys & 15) || ((uintptr_t)payload.data & 15)) return fail(TQ_EINVAL, "keys/payload not 16-byte aligned");
  if (payload.type != TQ_U8 && payload.type != TQ_I32 && payload.type != TQ_I64) return fail(TQ_EINVAL, "payload type");
  if (!nullable && (key_valid || payload.valid))
    return fail(TQ_EINVAL, "validity bitmaps on the key or payload: use tq_join_build_nullable");
  int64_t cap_max = cap_max_for_bytes(bytes);
  if (cap_max == 0) return fail(TQ_EINVAL, "table buffer of %zu bytes is too small", bytes);
  RowPlan P;
  tq_status s = make_plan(&P, filt, nfilt, p, np, nullptr, 0, nullptr, n, nullable);
  if (s) return s;
  TableHeader* h = static_cast<TableHeader*>(d_table);
  DCol pc = {payload.data, payload.type, payload.valid};
  const int64_t part_grid = std::max<int64_t>(1, (n + kPartRows - 1) / kPartRows);
  if (part_grid <= part_grid_max(cap_max)) {
    // the rows' segments fit the scratch area: partition, count, then fill regions (or CAS)
    TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_build_part<NC>, dim3((int)part_grid), dim3(kPartBlock), 0, stream,
                                                  P, d_keys, pc, n, h, cap_max, skip, flags, key_valid));
    hipLaunchKernelGGL(k_build_regions, dim3(kRegionBins), dim3(kFinBlock), 0, stream, h, cap_max, (int)part_grid,
                       load_factor, skip, flags, cap_rule(load_factor));
    // the fallback does nothing unless a region overflowed (rare: keys whose hashes
    // crowd one region) or the table is past the regions' range, which only a buffer
    // of more than 2^kMaxPassLog2Cap slots allows; for a smaller one a small grid
    // keeps the launch that finds nothing to do cheap (dispatching hundreds of
    // workgroups that return at once took about 4 us), for a larger one the grid is
    // sized for inserting every row
    const int fb_grid = cap_max > ((int64_t)1 << kMaxPassLog2Cap) ? stream_grid(n, 2) : kFallbackBlocks;
    TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_build_fallback<NC>, dim3(fb_grid), dim3(kBlock), 0,
                                                  stream, P, d_keys, pc, n, h, cap_max, key_valid));
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  const bool count = (np > 0 || (flags & TQ_SELECT_PARTITION) || key_valid) && n > 0;
  Range R = split_rows(std::max<int64_t>(n, 1), kMaxCountBlocks);
  // enough blocks to clear the tags quickly; blocks past the rows count zero
  const int64_t clear_blocks = std::min<int64_t>((cap_max >> kLog2Bucket) / kBlock, kMaxCountBlocks);
  const int count_grid = (int)std::max<int64_t>(R.nblk, clear_blocks);
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_build_count<NC>, dim3(count_grid), dim3(kBlock), 0, stream, P, d_keys, n,
                                                R.per, h, cap_max, (int)count, skip, flags, key_valid));
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_build_insert<NC>, dim3(stream_grid(n, 8)), dim3(kBlock), 0, stream, P,
                                                d_keys, pc, n, h, cap_max, count ? (int64_t)-1 : n, R.nblk, load_factor,
                                                skip, flags, key_valid));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

extern "C" {

tq_status tq_join_build(void* d_table, size_t bytes, const int64_t* d_keys, tq_col payload, int64_t n,
                        const tq_col* filt, int32_t nfilt, const tq_pred* p, int32_t np, double load_factor,
                        int32_t skip, uint32_t flags, hipStream_t stream) {
  return join_build(d_table, bytes, d_keys, nullptr, payload, n, filt, nfilt, p, np, load_factor, skip, flags, false,
                    stream);
}

tq_status tq_join_build_nullable(void* d_table, size_t bytes, const int64_t* d_keys, const uint8_t* d_key_valid,
                                 tq_col payload, int64_t n, const tq_col* filt, int32_t nfilt, const tq_pred* p,
                                 int32_t np, double load_factor, int32_t skip, uint32_t flags, hipStream_t stream) {
  return join_build(d_table, bytes, d_keys, d_key_valid, payload, n, filt, nfilt, p, np, load_factor, skip, flags, true,
                    stream);
}

tq_status tq_join_probe_nullable(const void* d_table, const int64_t* d_probe_keys, const uint8_t* d_key_valid,
                                 int64_t n, const tq_col* cols, int32_t ncol, const tq_pred* p, int32_t np,
                                 const tq_agg* agg, hipStream_t stream) {
  if (!d_table) return fail(TQ_EINVAL, "table is NULL");
  if (!agg) return fail(TQ_EINVAL, "the probe under NULLs aggregates: agg is NULL");
  if (n < 0) return fail(TQ_EINVAL, "n < 0");
  if (n > 0 && !d_probe_keys) return fail(TQ_EINVAL, "probe keys are NULL");
  if ((uintptr_t)d_probe_keys & 15) return fail(TQ_EINVAL, "probe keys not 16-byte aligned");
  RowPlan P;
  tq_status s = make_plan(&P, cols, ncol, p, np, agg->sums, agg->nsum, nullptr, n, true);
  if (s) return s;
  AggTarget T{};
  AggMode mode;
  size_t lds = 0;
  if ((s = make_target(agg->d_state, agg->domain, agg->nsum, &T, &mode, &lds, agg->nullable != 0))) return s;
  if (n == 0) return TQ_OK;
  dim3 grid(agg_grid(n)), block(kAggBlock);
  TQ_DISPATCH_AGG(mode, P.ncol, agg->nsum, M, NC, NE,
                  hipLaunchKernelGGL((k_probe_agg<M, NC, NE>), grid, block, lds, stream,
                                     static_cast<const TableHeader*>(d_table), d_probe_keys, n, P, T, d_key_valid));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_join_probe(const void* d_table, const int64_t* d_probe_keys, int64_t n, const tq_col* cols, int32_t ncol,
                        const tq_pred* p, int32_t np, int64_t* d_out_probe_row, int64_t* d_out_payload,
                        int64_t capacity, int64_t* d_out_count, const tq_agg* agg, hipStream_t stream) {
  if (agg && agg->nullable) return fail(TQ_EINVAL, "a nullable group-by state: use tq_join_probe_nullable");
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
    bool all64 = true;
    for (int c = 0; c < P.ncol; c++) all64 = all64 && P.col[c].w == 8;
    const int nq = ne_bucket(agg->nsum);
    const size_t agg_lds16 = (lds + 15) / 16 * 16;
    const size_t pipe_lds = agg_lds16 + (size_t)(kAggBlock / kWave) * kPipeQ * 4;
    const size_t bloom_lds = agg_lds16 + (size_t)(kBloomPipeBlock / kWave) * kPipeQ * 4;
    if (all64 && nq <= 2 && pipe_lds <= kMaxPipeLds) {
      // with the build's Bloom filter in LDS when it fits beside the queues and
      // the group-by (one workgroup of 16 waves per CU), else without (two of 8)
      const bool bloom = bloom_lds <= kMaxBloomPipeLds;
      const int threads = bloom ? kBloomPipeBlock : kAggBlock;
      const int agg_lds = (int)agg_lds16;
      UnitPlan U;
      const bool fast = mode == kDense && P.np == 0 && P.ncol <= 2 && unit_plan(P, &U);
      // one launch per kPipeMaxRows rows (an even count: the 16-byte column loads stay aligned)
      for (int64_t c0 = 0; c0 < n; c0 += kPipeMaxRows) {
        const int64_t nc = std::min<int64_t>(kPipeMaxRows, n - c0);
        RowPlan Pc = P;
        for (int c = 0; c < Pc.ncol; c++) Pc.col[c].p = static_cast<const int64_t*>(P.col[c].p) + c0;
        const int64_t want = (nc + (int64_t)threads * kPipeRows - 1) / ((int64_t)threads * kPipeRows);
        const int64_t cap = std::min<int64_t>(kAggRows, (int64_t)(bloom ? 1 : kPipeBlocksPerCU) * device_cu_count());
        dim3 grid((int)std::max<int64_t>(1, std::min(want, cap))), block(threads);
        TQ_DISPATCH_AGG(mode, P.ncol, agg->nsum, M, NC, NE, if constexpr (NE <= 2) {
          const size_t q = (size_t)(threads / kWave) * kPipeQ * 4;
          bool launched = false;
          if constexpr (M == kDense && NC <= 2 && NE == 1) {  // (two sums would spill registers to memory)
            if (fast) {
              if (bloom)
                hipLaunchKernelGGL((k_probe_compact<NC, NE>), grid, block, agg_lds + q, stream, h, d_probe_keys + c0,
                                   nc, Pc, T, U, agg_lds);
              else
                hipLaunchKernelGGL((k_probe_pipe<M, NC, NE, false, true>), grid, block, agg_lds + q, stream, h,
                                   d_probe_keys + c0, nc, Pc, T, U, agg_lds);
              launched = true;
            }
          }
          if (!launched) {
            if (bloom)
              hipLaunchKernelGGL((k_probe_pipe<M, NC, NE, true, false>), grid, block, agg_lds + q, stream, h,
                                 d_probe_keys + c0, nc, Pc, T, U, agg_lds);
            else
              hipLaunchKernelGGL((k_probe_pipe<M, NC, NE, false, false>), grid, block, agg_lds + q, stream, h,
                                 d_probe_keys + c0, nc, Pc, T, U, agg_lds);
          }
        });
      }
    } else {
      dim3 grid(agg_grid(n)), block(kAggBlock);
      TQ_DISPATCH_AGG(mode, P.ncol, agg->nsum, M, NC, NE,
                      hipLaunchKernelGGL((k_probe_agg<M, NC, NE>), grid, block, lds, stream, h, d_probe_keys, n, P, T,
                                         nullptr));
    }
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
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_probe_count<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, h, d_probe_keys, n,
                                              R.per, P, cnt));
  hipLaunchKernelGGL(k_scan_blocks<0>, dim3(1), dim3(1024), 0, stream, cnt, R.nblk, d_out_count);
  TQ_DISPATCH_NC(P.ncol, NC, hipLaunchKernelGGL(k_probe_write<NC>, dim3(R.nblk), dim3(kBlock), 0, stream, h, d_probe_keys, n,
                                              R.per, P, cnt, d_out_probe_row, d_out_payload, capacity));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
