// Batched join + group-by instances: one queue launch per phase.
//
// Work area: WorkHeader | BInst[n] | int64 ctr[n][kCtr] | uint64 item[n_items] |
// uint32 bloom[...] (each instance's Bloom filter of its kept build keys).
// An item is (type, instance, index). The list holds every build tile, then
// every probe tile, then the finalize items (single-chunk finalizes and chunk
// counts), then the chunk writes; each group is one phase. Every phase is one
// persistent launch whose workgroups take items from the phase's range of the
// list through an atomic cursor; an item depends only on items of earlier
// phases, which the launch boundary has completed and made visible, so no
// workgroup ever waits for another.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "groupby.h"
#include "table.h"

namespace tq {
namespace {

constexpr int kBBlock = 512;
constexpr int kFinChunk = 8192;  // keys per finalize chunk
constexpr int kMaxChunks = 8;    // domain <= 65536
constexpr int kCtr = 16;         // counters per instance: chunk counts at [8..16)
constexpr int kPhases = 4;       // build, probe, finalize (single chunk or chunk counts), chunk writes
constexpr int kBPR = 2;          // rows per lane in probe items
constexpr int kBuildQ = 2 * 64;  // a build item's per-wave queue of kept rows (at most 63 + 64)
constexpr int kMinBloomWords = 64;    // an instance's filter: 2 bits per build row, 256 B to 32 KiB
constexpr int kMaxBloomWords = 8192;

enum ItemType { kItBuild = 0, kItProbe = 1, kItFinOne = 2, kItFinCount = 3, kItFinWrite = 4 };

__host__ __device__ inline uint64_t make_item(int type, int64_t inst, int64_t idx) {
  return ((uint64_t)type << 60) | ((uint64_t)inst << 36) | (uint64_t)idx;
}

struct BInst {
  const void* dcol[4];
  const void* fcol[4];
  int64_t n_dim, n_fact, domain;
  void* table;
  int64_t cap_max;
  int32_t log2cap, build_tile, probe_tile, nchunks;
  int64_t n_build_items, n_probe_items;
  void* state;
  uint32_t* bloom;  // the instance's filter (bloom_nw words, a power of two)
  int32_t bloom_nw;
  int64_t* keys;
  int64_t* count;
  int64_t* sums;
  double* avg;
  int64_t* ngroups;
};

struct WorkHeader {
  int64_t head[kPhases];  // next item of each phase
  int64_t end[kPhases];   // the phase's items are [end[p - 1], end[p])
  int64_t n_items;
  int32_t n_inst;
  int32_t err;
};
static_assert(sizeof(WorkHeader) <= 256, "header");

struct BQuery {
  int32_t dtype[4];
  int32_t ndim;
  DPred pred[2];
  int32_t np;
  int32_t ftype[4];
  int32_t nfact;
  DExpr sums[2];
  int32_t nsum;
  uint32_t flags;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
  size_t inst_off, item_off, ctr_off, bloom_off, bytes;
};

Layout layout(int32_t n, int64_t n_items, int64_t bloom_words = 0) {
  Layout L;
  L.inst_off = 256;
  L.ctr_off = L.inst_off + al((size_t)n * sizeof(BInst));
  L.item_off = L.ctr_off + al((size_t)n * kCtr * 8);
  L.bloom_off = L.item_off + al((size_t)n_items * 8);
  L.bytes = L.bloom_off + al((size_t)bloom_words * 4);
  return L;
}

// Filter words of an instance with n_dim build rows.
int32_t bloom_words_for(int64_t n_dim) {
  int64_t w = kMinBloomWords;
  while (w < kMaxBloomWords && w * 16 < n_dim) w *= 2;
  return (int32_t)w;
}

int64_t count_bloom_words(const tq_instance* h, int32_t n) {
  int64_t t = 0;
  for (int i = 0; i < n; i++) t += bloom_words_for(h[i].n_dim);
  return t;
}

// The filter's word (from hash bits 41.., above those of bloom_bits) for a
// key's multiplicative hash.
__device__ __forceinline__ uint32_t inst_bloom_word(uint64_t hh, int32_t nw) {
  return (uint32_t)(hh >> 41) & (uint32_t)(nw - 1);
}

int log2cap_for_rows(int64_t rows, double lf) {
  double need = ceil((double)rows / lf);
  int l = 6;
  while (l < 62 && (double)((int64_t)1 << l) < need) l++;
  return l;
}

int64_t cap_max_for(size_t bytes) {
  int64_t cap = 0;
  for (int l = 6; l < 62; l++) {
    int64_t c = (int64_t)1 << l;
    size_t need = kHeaderBytes + (size_t)kMaxPartBlocks * 8 + table_tag_bytes(c) + (size_t)c * 16;
    if (need > bytes) break;
    cap = c;
  }
  return cap;
}

int64_t count_items(const tq_instance* h, int32_t n) {
  int64_t t = 0;
  for (int i = 0; i < n; i++) {
    t += (h[i].n_dim + h[i].build_tile - 1) / h[i].build_tile;
    t += (h[i].n_fact + h[i].probe_tile - 1) / h[i].probe_tile;
    int64_t ch = (h[i].domain + kFinChunk - 1) / kFinChunk;
    t += ch == 1 ? 1 : 2 * ch;
  }
  return t;
}

__global__ __launch_bounds__(256) void k_batched_prep(WorkHeader* hdr, const BInst* insts, int64_t* ctrs, int32_t n,
                                                      int32_t nsum, uint32_t flags) {
  if (blockIdx.x == 0 && threadIdx.x < kPhases) hdr->head[threadIdx.x] = threadIdx.x == 0 ? 0 : hdr->end[threadIdx.x - 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->err = 0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BInst& I = insts[i];
    if (threadIdx.x < kCtr) ctrs[(int64_t)i * kCtr + threadIdx.x] = 0;
    TableHeader* th = static_cast<TableHeader*>(I.table);
    if (threadIdx.x == 0) {
      th->magic = kTableMagic;
      th->err = 0;
      th->cap_max = I.cap_max;
      th->log2cap = I.log2cap;
      th->skip = 0;
      th->n = I.n_dim;
      th->nblk = 0;
      th->flags = flags;
      th->lf = 0;
      th->log2g = I.log2cap - kLog2Bucket;
      th->regions = 0;
      th->alt = 0;
      th->ovf = 0;
      th->bloom_log2w = 0;
      StateHeader* sh = static_cast<StateHeader*>(I.state);
      sh->magic = kStateMagic;
      sh->err = 0;
      sh->domain = I.domain;
      sh->nsum = nsum;
      sh->rows = 1;
      sh->used = 0;
    }
    v4i32* tags = reinterpret_cast<v4i32*>(table_tags(th));
    const v4i32 z = {0, 0, 0, 0};
    for (int64_t g = threadIdx.x; g < ((int64_t)1 << I.log2cap) / kBucket; g += blockDim.x) tags[g] = z;
    int64_t* d = state_data(I.state);
    for (int64_t e = threadIdx.x; e < I.domain * (1 + nsum); e += blockDim.x) d[e] = 0;
    for (int e = threadIdx.x; e < I.bloom_nw; e += blockDim.x) I.bloom[e] = 0u;
  }
}

// Compaction of keys [k_lo, k_hi) of a rows=1 state into the outputs at `base`; returns the live count.
__device__ int64_t fin_write(const BInst& I, int nsum, int64_t k_lo, int64_t k_hi, int64_t base, int64_t* ws) {
  const int stride = 1 + nsum;
  const int64_t* d = state_data(I.state);
  for (int64_t k0 = k_lo; k0 < k_hi; k0 += blockDim.x) {
    int64_t k = k0 + threadIdx.x;
    int64_t e[3] = {0, 0, 0};
    bool live = false;
    if (k < k_hi) {
#pragma unroll
      for (int j = 0; j < 3; j++)
        if (j < stride) e[j] = d[k * stride + j];
      live = e[0] != 0;
    }
    int64_t excl;
    int64_t tot = block_excl_scan(live ? 1 : 0, &excl, ws);
    if (live) {
      int64_t g = base + excl;
      I.keys[g] = k;
      I.count[g] = e[0];
#pragma unroll
      for (int j = 0; j < 2; j++) {
        if (j < nsum) {
          I.sums[g * nsum + j] = e[1 + j];
          I.avg[g * nsum + j] = (double)e[1 + j] / (double)e[0];
        }
      }
    }
    base += tot;
  }
  return base;
}

__device__ int64_t fin_count(const BInst& I, int nsum, int64_t k_lo, int64_t k_hi, int64_t* ws) {
  const int stride = 1 + nsum;
  const int64_t* d = state_data(I.state);
  int64_t c = 0;
  for (int64_t k = k_lo + threadIdx.x; k < k_hi; k += blockDim.x) c += d[k * stride] != 0;
  return block_sum(c, ws);
}

template <int MODE>
__device__ void probe_item(const BQuery& Q, const BInst& I, int64_t idx, char* smem, int32_t* err) {
  AggTarget T;
  T.hdr = static_cast<const StateHeader*>(I.state);
  T.data = state_data(I.state);
  T.err = &static_cast<StateHeader*>(I.state)->err;
  T.domain = I.domain;
  T.stride = 1 + Q.nsum;
  T.rows = 1;
  size_t lds;
  agg_mode(I.domain, T.stride, &T.log2hcap, &lds);
  LdsAgg<MODE> agg;
  agg.defer = true;  // a key outside the domain is remembered and latched below
  agg.init(T, smem);
  // the instance's filter, after the partials: most probe rows have no
  // partner, and a row it rejects loads nothing from the table
  uint32_t* bloom = reinterpret_cast<uint32_t*>(smem + kLdsAggBytes);
  const int32_t nw = I.bloom_nw;
  for (int e = threadIdx.x; e < nw; e += blockDim.x) bloom[e] = I.bloom[e];
  __syncthreads();
  const TableHeader* th = static_cast<const TableHeader*>(I.table);
  Probe pr;
  pr.setup(th);
  const int64_t lo = idx * I.probe_tile, hi = min(I.n_fact, lo + I.probe_tile);
  DCol fc[4];
#pragma unroll
  for (int c = 0; c < 4; c++) fc[c] = DCol{I.fcol[c] ? I.fcol[c] : I.fcol[0], Q.ftype[c] ? Q.ftype[c] : 8};
  // the columns of a lane's next rows are requested while its current rows
  // walk the table (right after their first tag loads are issued)
  int64_t vn[4][kBPR];
  auto load = [&](int64_t r) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
      if (c < Q.nfact) load4<kBPR>(fc[c], r, r + kBPR <= hi, hi, vn[c]);
      else {
#pragma unroll
        for (int i = 0; i < kBPR; i++) vn[c][i] = 0;
      }
    }
  };
  const int64_t step = (int64_t)blockDim.x * kBPR;
  int64_t r0 = lo + (int64_t)threadIdx.x * kBPR;
  if (r0 < hi) load(r0);
  for (; r0 < hi; r0 += step) {
    int64_t k[kBPR], e[kBPR][2];
    bool ok[kBPR];
#pragma unroll
    for (int i = 0; i < kBPR; i++) {
      k[i] = vn[0][i];
      const uint64_t hh = mulhash(k[i]);
      const uint32_t m = bloom_bits(hh);
      ok[i] = r0 + i < hi && (bloom[inst_bloom_word(hh, nw)] & m) == m;
#pragma unroll
      for (int j = 0; j < 2; j++) e[i][j] = j < Q.nsum ? eval_expr<4, kBPR>(Q.sums[j], vn, i) : 0;
    }
    const int64_t r1 = r0 + step;
    pr.walk(
        ok, k,
        [&](const bool (&hit)[kBPR], const int64_t (&pay)[kBPR]) {
#pragma unroll
          for (int i = 0; i < kBPR; i++)
            if (hit[i]) agg.add(T, pay[i], e[i], Q.nsum);
        },
        [&] {
          if (r1 < hi) load(r1);
        });
  }
  // a group key outside the instance's domain: latched in the instance's state
  // (by flush) and in the work area, where tq_batched_check finds it
  if (__syncthreads_or(agg.bad) && threadIdx.x == 0) latch_error(err, TQ_EDOMAIN);
  agg.flush(T);
}

// One launch per phase, instantiated per phase so that each holds only the
// code of its own items: a kernel with every phase's code is allocated the
// registers of the largest (148 VGPRs, one workgroup per CU).
template <int PHASE>
__global__ __launch_bounds__(kBBlock) void k_batched(BQuery Q, WorkHeader* hdr, const BInst* insts,
                                                      const uint64_t* items, int64_t* ctrs) {
  constexpr int phase = PHASE;
  extern __shared__ __align__(16) char smem[];
  __shared__ uint64_t s_item;
  __shared__ int64_t s_base;
  __shared__ int64_t ws[kBBlock / kWave];
  const int64_t end = hdr->end[phase];
  for (;;) {
    if (threadIdx.x == 0) {
      int64_t i = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&hdr->head[phase]), 1ull);
      s_item = i < end ? items[i] : ~0ull;
    }
    __syncthreads();
    const uint64_t it = s_item;
    __syncthreads();
    if (it == ~0ull) break;
    const int type = (int)(it >> 60);
    const int64_t inst = (int64_t)((it >> 36) & 0xffffffull);
    const int64_t idx = (int64_t)(it & 0xfffffffffull);
    const BInst& I = insts[inst];
    int64_t* ctr = ctrs + inst * kCtr;

    if (PHASE == 0 && type == kItBuild) {
      // The rows that pass the predicates (most do not) are compacted per
      // wave into an LDS queue of (key, payload) and inserted 64 at a time,
      // one per lane, with the instance's filter bits: each CAS round then
      // works on a full wave of rows instead of a few lanes of four.
      const TableHeader* th = static_cast<const TableHeader*>(I.table);
      uint32_t* words = table_tags(const_cast<TableHeader*>(th));
      v2i64* slots = reinterpret_cast<v2i64*>(table_slots(const_cast<TableHeader*>(th), I.cap_max));
      const int64_t lo = idx * I.build_tile, hi = min(I.n_dim, lo + I.build_tile);
      const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
      v2i64* bq = reinterpret_cast<v2i64*>(smem) + wave * kBuildQ;  // this wave's queue
      int qn = 0;  // queued rows (the same in every lane)
      auto insert_queued = [&](int cnt) {  // entries [0, cnt), cnt <= 64
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        bool pend[1] = {lane < cnt};
        const v2i64 e = pend[0] ? bq[lane] : v2i64{0, 0};
        int64_t k1[1] = {e.x}, p1[1] = {e.y};
        if (pend[0]) {
          const uint64_t hh = mulhash(k1[0]);
          atomicOr(&I.bloom[inst_bloom_word(hh, I.bloom_nw)], bloom_bits(hh));
        }
        table_insert<1>(words, slots, I.log2cap, 0, pend, k1, p1);
      };
      DCol dc[4];
#pragma unroll
      for (int c = 0; c < 4; c++) dc[c] = DCol{I.dcol[c] ? I.dcol[c] : I.dcol[0], Q.dtype[c] ? Q.dtype[c] : 8};
      // the loop runs alike in every lane of a wave (lanes past the tile hold no rows)
      for (int64_t wb = lo + (int64_t)wave * kWave * kRows; wb < hi; wb += (int64_t)blockDim.x * kRows) {
        const int64_t r0 = wb + (int64_t)lane * kRows;
        const bool full = r0 + kRows <= hi;
        int64_t v[4][kRows];
#pragma unroll
        for (int c = 0; c < 4; c++) {
          if (c < Q.ndim && r0 < hi) load4(dc[c], r0, full, hi, v[c]);
          else {
#pragma unroll
            for (int i = 0; i < kRows; i++) v[c][i] = 0;
          }
        }
#pragma unroll
        for (int i = 0; i < kRows; i++) {
          // at most two predicates, read from the query directly (a plan copied
          // into a local structure and indexed in a loop lives in scratch memory)
          bool ok = r0 + i < hi;
#pragma unroll
          for (int j = 0; j < 2; j++) {
            if (j < Q.np) {
              const int64_t x = pick<4, kRows>(v, i, Q.pred[j].mask);
              ok = ok && x >= Q.pred[j].lo && x <= Q.pred[j].hi;
            }
          }
          const uint64_t m = __ballot(ok);
          if (ok) bq[qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
              v2i64{v[0][i], v[1][i]};
          qn += __builtin_popcountll(m);
          if (qn >= kWave) {
            insert_queued(kWave);
            // the rest (fewer than 64) moves to the front
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const bool mv = lane < qn - kWave;
            const v2i64 t = mv ? bq[kWave + lane] : v2i64{0, 0};
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (mv) bq[lane] = t;
            qn -= kWave;
          }
        }
      }
      if (qn > 0) insert_queued(qn);
    } else if (PHASE == 1 && type == kItProbe) {
      if (I.domain * (1 + Q.nsum) * 8 <= kLdsAggBytes) probe_item<kDense>(Q, I, idx, smem, &hdr->err);
      else probe_item<kHash>(Q, I, idx, smem, &hdr->err);
    } else if (PHASE == 2 && type == kItFinOne) {
      int64_t g = fin_write(I, Q.nsum, 0, I.domain, 0, ws);
      if (threadIdx.x == 0) *I.ngroups = g;
    } else if (PHASE == 2 && type == kItFinCount) {
      int64_t c = fin_count(I, Q.nsum, idx * kFinChunk, min(I.domain, (idx + 1) * kFinChunk), ws);
      if (threadIdx.x == 0) ctr[8 + idx] = c;
    } else if (PHASE == 3 && type == kItFinWrite) {
      if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int64_t c = 0; c < idx; c++) b += ctr[8 + c];
        s_base = b;
      }
      __syncthreads();
      int64_t g = fin_write(I, Q.nsum, idx * kFinChunk, min(I.domain, (idx + 1) * kFinChunk), s_base, ws);
      if (threadIdx.x == 0 && idx == I.nchunks - 1) *I.ngroups = g;
    }
    __syncthreads();
  }
}

tq_status make_query(const tq_batch_query* q, BQuery* Q) {
  memset(Q, 0, sizeof *Q);
  if (!q) return fail(TQ_EINVAL, "query is NULL");
  if (q->ndim < 2 || q->ndim > 4 || q->nfact < 1 || q->nfact > 4) return fail(TQ_EINVAL, "column counts");
  if (q->np < 0 || q->np > 2 || q->nsum < 0 || q->nsum > 2) return fail(TQ_EINVAL, "predicate or sum count");
  if (q->dim_types[0] != TQ_I64 || q->fact_types[0] != TQ_I64) return fail(TQ_EINVAL, "keys must be int64");
  for (int c = 0; c < 4; c++) {
    if (c < q->ndim && q->dim_types[c] != TQ_U8 && q->dim_types[c] != TQ_I32 && q->dim_types[c] != TQ_I64)
      return fail(TQ_EINVAL, "dimension column %d type", c);
    if (c < q->nfact && q->fact_types[c] != TQ_U8 && q->fact_types[c] != TQ_I32 && q->fact_types[c] != TQ_I64)
      return fail(TQ_EINVAL, "fact column %d type", c);
    Q->dtype[c] = c < q->ndim ? q->dim_types[c] : 0;
    Q->ftype[c] = c < q->nfact ? q->fact_types[c] : 0;
  }
  Q->ndim = q->ndim;
  Q->nfact = q->nfact;
  Q->np = q->np;
  for (int j = 0; j < q->np; j++) {
    if (q->preds[j].col < 0 || q->preds[j].col >= q->ndim) return fail(TQ_EINVAL, "predicate column");
    Q->pred[j] = DPred{1u << q->preds[j].col, q->preds[j].lo, q->preds[j].hi};
  }
  Q->nsum = q->nsum;
  for (int j = 0; j < q->nsum; j++) {
    if (q->sums[j].nf < 1 || q->sums[j].nf > 3) return fail(TQ_EINVAL, "sum factors");
    Q->sums[j].nf = q->sums[j].nf;
    for (int f = 0; f < q->sums[j].nf; f++) {
      const tq_factor& F = q->sums[j].f[f];
      if (F.col < -1 || F.col >= q->nfact) return fail(TQ_EINVAL, "sum column");
      Q->sums[j].f[f] = make_factor(F.col, F.sign, F.add);
    }
  }
  if (q->join_flags & ~TQ_UNIQUE_KEYS) return fail(TQ_EINVAL, "join_flags: only TQ_UNIQUE_KEYS applies to batched instances");
  Q->flags = q->join_flags;
  return TQ_OK;
}

}  // namespace
}  // namespace tq

using namespace tq;

extern "C" {

size_t tq_batched_state_bytes(int64_t domain, int32_t nsum) {
  if (domain <= 0 || nsum < 0 || nsum > 2) return 0;
  size_t shared = kHeaderBytes + (size_t)domain * (1 + nsum) * 8;
  return std::max(shared, tq_groupby_state_bytes(domain, nsum));  // also fits the stand-alone layout
}

size_t tq_batched_work_bytes(const tq_instance* h, int32_t n) {
  if (!h || n <= 0) return 0;
  for (int i = 0; i < n; i++)
    if (h[i].build_tile <= 0 || h[i].probe_tile <= 0) return 0;
  return layout(n, count_items(h, n), count_bloom_words(h, n)).bytes;
}

tq_status tq_batched_prepare(const tq_batch_query* q, const tq_instance* h, int32_t n, void* d_work, size_t work_bytes,
                             hipStream_t stream) {
  BQuery Q;
  tq_status s = make_query(q, &Q);
  if (s) return s;
  if (!h || n <= 0 || n > (1 << 24) || !d_work) return fail(TQ_EINVAL, "instances");
  std::vector<BInst> bi((size_t)n);
  std::vector<uint64_t> items;
  for (int i = 0; i < n; i++) {
    const tq_instance& x = h[i];
    if (x.n_dim < 0 || x.n_fact < 0 || x.domain <= 0 || x.domain > (int64_t)kFinChunk * kMaxChunks)
      return fail(TQ_EINVAL, "instance %d: sizes or domain (<= 65536)", i);
    if (x.build_tile < 64 || x.probe_tile < 64 || x.build_tile % 64 || x.probe_tile % 64)
      return fail(TQ_EINVAL, "instance %d: tiles must be multiples of 64", i);
    if (!(x.load_factor > 0 && x.load_factor <= 0.9)) return fail(TQ_EINVAL, "instance %d: load factor", i);
    for (int c = 0; c < 4; c++) {
      if (c < q->ndim && ((!x.dim_cols[c] && x.n_dim) || ((uintptr_t)x.dim_cols[c] & 15)))
        return fail(TQ_EINVAL, "instance %d: dimension column %d", i, c);
      if (c < q->nfact && ((!x.fact_cols[c] && x.n_fact) || ((uintptr_t)x.fact_cols[c] & 15)))
        return fail(TQ_EINVAL, "instance %d: fact column %d", i, c);
    }
    if (!x.d_table || !x.d_state || !x.d_keys || !x.d_count || !x.d_sums || !x.d_avg || !x.d_ngroups)
      return fail(TQ_EINVAL, "instance %d: NULL buffer", i);
    if (x.state_bytes < tq_batched_state_bytes(x.domain, q->nsum)) return fail(TQ_EINVAL, "instance %d: state size", i);
    BInst& b = bi[(size_t)i];
    memset(&b, 0, sizeof b);
    for (int c = 0; c < 4; c++) {
      b.dcol[c] = c < q->ndim ? x.dim_cols[c] : nullptr;
      b.fcol[c] = c < q->nfact ? x.fact_cols[c] : nullptr;
    }
    b.n_dim = x.n_dim;
    b.n_fact = x.n_fact;
    b.domain = x.domain;
    b.table = x.d_table;
    b.cap_max = cap_max_for(x.table_bytes);
    b.log2cap = log2cap_for_rows(x.n_dim, x.load_factor);
    if (b.cap_max == 0 || ((int64_t)1 << b.log2cap) > b.cap_max) return fail(TQ_EINVAL, "instance %d: table too small", i);
    b.build_tile = x.build_tile;
    b.probe_tile = x.probe_tile;
    b.nchunks = (int32_t)((x.domain + kFinChunk - 1) / kFinChunk);
    b.n_build_items = (x.n_dim + x.build_tile - 1) / x.build_tile;
    b.n_probe_items = (x.n_fact + x.probe_tile - 1) / x.probe_tile;
    b.state = x.d_state;
    b.keys = x.d_keys;
    b.count = x.d_count;
    b.sums = x.d_sums;
    b.avg = x.d_avg;
    b.ngroups = x.d_ngroups;
  }
  int64_t end[kPhases];
  for (int i = 0; i < n; i++)
    for (int64_t t = 0; t < bi[(size_t)i].n_build_items; t++) items.push_back(make_item(kItBuild, i, t));
  end[0] = (int64_t)items.size();
  for (int i = 0; i < n; i++)
    for (int64_t t = 0; t < bi[(size_t)i].n_probe_items; t++) items.push_back(make_item(kItProbe, i, t));
  end[1] = (int64_t)items.size();
  for (int i = 0; i < n; i++) {
    if (bi[(size_t)i].nchunks == 1) items.push_back(make_item(kItFinOne, i, 0));
    else
      for (int c = 0; c < bi[(size_t)i].nchunks; c++) items.push_back(make_item(kItFinCount, i, c));
  }
  end[2] = (int64_t)items.size();
  for (int i = 0; i < n; i++)
    if (bi[(size_t)i].nchunks > 1)
      for (int c = 0; c < bi[(size_t)i].nchunks; c++) items.push_back(make_item(kItFinWrite, i, c));
  end[3] = (int64_t)items.size();
  Layout L = layout(n, (int64_t)items.size(), count_bloom_words(h, n));
  {
    uint32_t* bw = reinterpret_cast<uint32_t*>(static_cast<char*>(d_work) + L.bloom_off);
    for (int i = 0; i < n; i++) {
      bi[(size_t)i].bloom = bw;
      bi[(size_t)i].bloom_nw = bloom_words_for(h[i].n_dim);
      bw += bi[(size_t)i].bloom_nw;
    }
  }
  if (work_bytes < L.bytes) return fail(TQ_EINVAL, "work area has %zu bytes, needs %zu", work_bytes, L.bytes);
  WorkHeader wh;
  memset(&wh, 0, sizeof wh);
  for (int p = 0; p < kPhases; p++) {
    wh.end[p] = end[p];
    wh.head[p] = p == 0 ? 0 : end[p - 1];
  }
  wh.n_items = (int64_t)items.size();
  wh.n_inst = n;
  char* w = static_cast<char*>(d_work);
  TQ_HIP(hipMemcpyAsync(w, &wh, sizeof wh, hipMemcpyHostToDevice, stream));
  TQ_HIP(hipMemcpyAsync(w + L.inst_off, bi.data(), bi.size() * sizeof(BInst), hipMemcpyHostToDevice, stream));
  TQ_HIP(hipMemcpyAsync(w + L.item_off, items.data(), items.size() * 8, hipMemcpyHostToDevice, stream));
  TQ_HIP(hipStreamSynchronize(stream));
  return TQ_OK;
}

tq_status tq_batched_run(const tq_batch_query* q, void* d_work, int32_t n, hipStream_t stream) {
  BQuery Q;
  tq_status s = make_query(q, &Q);
  if (s) return s;
  if (!d_work || n <= 0) return fail(TQ_EINVAL, "work area or instance count");
  Layout L = layout(n, 0);  // the item list is last; the kernel reads its length from the header
  char* w = static_cast<char*>(d_work);
  auto* hdr = reinterpret_cast<WorkHeader*>(w);
  auto* insts = reinterpret_cast<const BInst*>(w + L.inst_off);
  auto* items = reinterpret_cast<const uint64_t*>(w + L.item_off);
  auto* ctrs = reinterpret_cast<int64_t*>(w + L.ctr_off);
  hipLaunchKernelGGL(k_batched_prep, dim3(std::min(n, 8192)), dim3(256), 0, stream, hdr, insts, ctrs, n, Q.nsum,
                     Q.flags);
  TQ_HIP(hipGetLastError());
  static_assert(kPhases == 4, "one kernel per phase");
  void (*kern[kPhases])(BQuery, WorkHeader*, const BInst*, const uint64_t*, int64_t*) = {
      k_batched<0>, k_batched<1>, k_batched<2>, k_batched<3>};
  for (int p = 0; p < kPhases; p++) {
    int per_cu = 0;
    const size_t lds = kLdsAggBytes + (p == 1 ? (size_t)kMaxBloomWords * 4 : 0);  // probe items: the filter too
    TQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern[p], kBBlock, lds));
    per_cu = std::max(1, std::min(per_cu, 4));
    hipLaunchKernelGGL(kern[p], dim3(device_cu_count() * per_cu), dim3(kBBlock), lds, stream, Q, hdr, insts,
                       items, ctrs);
  }
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_batched_check(const void* d_work, hipStream_t stream) {
  if (!d_work) return fail(TQ_EINVAL, "work area is NULL");
  TQ_HIP(hipStreamSynchronize(stream));
  WorkHeader wh;
  TQ_HIP(hipMemcpy(&wh, d_work, sizeof wh, hipMemcpyDeviceToHost));
  if (wh.err) return fail(wh.err, "a batched work item latched an error");
  return TQ_OK;
}

tq_status tq_batched_run_per_instance(const tq_batch_query* q, const tq_instance* h, int32_t n, hipStream_t stream) {
  BQuery Q;
  tq_status s = make_query(q, &Q);
  if (s) return s;
  for (int i = 0; i < n; i++) {
    const tq_instance& x = h[i];
    tq_col dcols[4] = {}, fcols[4] = {};
    for (int c = 0; c < 4; c++) {
      dcols[c] = tq_col{x.dim_cols[c], q->dim_types[c]};
      fcols[c] = tq_col{x.fact_cols[c], q->fact_types[c]};
    }
    if ((s = tq_join_table_init(x.d_table, x.table_bytes, stream))) return s;
    if ((s = tq_join_build(x.d_table, x.table_bytes, static_cast<const int64_t*>(x.dim_cols[0]), dcols[1], x.n_dim,
                           dcols, q->ndim, q->preds, q->np, x.load_factor, 0, q->join_flags, stream)))
      return s;
    if ((s = tq_groupby_init(x.d_state, x.state_bytes, x.domain, q->nsum, stream))) return s;
    tq_agg agg{x.d_state, x.domain, q->sums, q->nsum};
    if ((s = tq_join_probe(x.d_table, static_cast<const int64_t*>(x.fact_cols[0]), x.n_fact, fcols, q->nfact, nullptr, 0,
                           nullptr, nullptr, 0, nullptr, &agg, stream)))
      return s;
    if ((s = tq_groupby_finalize(x.d_state, x.d_keys, x.d_count, x.d_sums, x.d_avg, x.d_ngroups, stream))) return s;
  }
  return TQ_OK;
}

}  // extern "C"
