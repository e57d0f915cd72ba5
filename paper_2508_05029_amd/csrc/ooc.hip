// Out-of-core partitioned join + aggregate over page-pool batches.
//
//   pass 1  stream the dimension (filter, hash partition) and the fact table
//           (hash partition) from pool pages; append each partition's slice
//           of every batch to that partition's holder, a list of fixed-size
//           device chunks reserved from the budget
//   spill   when a chunk cannot be reserved, chunks of the partition that
//           pass 2 reaches last are copied to pool pages on a stream of
//           their own and returned to the arena once the copy is done
//   pass 2  for p = 0, 1, ...: reload p's spilled chunks (and those of p + 1
//           ahead of use), gather p's dimension rows, build the table, probe
//           it with each fact chunk of p into the group-by state
//
// Holder chunk layout: R rows per chunk, column j of the side at byte offset
// off[j] (256-byte aligned), so that every chunk can be probed in place.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <vector>

#include "common.h"

namespace tq {
namespace {

constexpr size_t kAlign = 256;
constexpr int kSpillBatch = 8;     // chunks spilled per shortage
constexpr int kPrefetchParts = 3;  // pass 2 reloads this many partitions ahead of the one it joins, waiting if needed
size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct CopyDesc {
  const void* src;
  void* dst;
  int64_t n;  // elements
  int32_t w;  // element bytes
  int32_t pad;
};

// Copies a list of contiguous byte ranges: workgroup (x, y) copies the 16 KiB
// tiles x, x + gridDim.x, ... of range y, with the widest access that both of
// its pointers allow (tile starts keep the ranges' alignment).
constexpr int64_t kCopyTile = 16384;
typedef int v4i32 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_gather_copy(const CopyDesc* d) {
  const CopyDesc c = d[blockIdx.y];
  const int64_t bytes = c.n * c.w;
  const uintptr_t al = reinterpret_cast<uintptr_t>(c.src) | reinterpret_cast<uintptr_t>(c.dst);
  for (int64_t b0 = (int64_t)blockIdx.x * kCopyTile; b0 < bytes; b0 += (int64_t)gridDim.x * kCopyTile) {
    const int64_t nb = std::min<int64_t>(bytes - b0, kCopyTile);
    const char* s = static_cast<const char*>(c.src) + b0;
    char* o = static_cast<char*>(c.dst) + b0;
    int64_t j0 = 0;
    if ((al & 15) == 0) {
      const int64_t nv = nb >> 4;
      for (int64_t j = threadIdx.x; j < nv; j += 256)
        reinterpret_cast<v4i32*>(o)[j] = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(s) + j);
      j0 = nv << 4;
    } else if ((al & 7) == 0) {
      const int64_t nv = nb >> 3;
      for (int64_t j = threadIdx.x; j < nv; j += 256)
        reinterpret_cast<int64_t*>(o)[j] = reinterpret_cast<const int64_t*>(s)[j];
      j0 = nv << 3;
    } else if ((al & 3) == 0) {
      const int64_t nv = nb >> 2;
      for (int64_t j = threadIdx.x; j < nv; j += 256)
        reinterpret_cast<int32_t*>(o)[j] = reinterpret_cast<const int32_t*>(s)[j];
      j0 = nv << 2;
    }
    for (int64_t j = j0 + threadIdx.x; j < nb; j += 256) o[j] = s[j];
  }
}

struct ChunkRef {
  int64_t dev = -1;  // arena chunk id, or -1 when not resident
  int32_t page = -1, sub = -1;  // spill location
  int64_t rows = 0;
  bool pinned = false;  // an append that is being assembled writes into it
};

struct Holder {
  std::vector<ChunkRef> chunks;
  int64_t rows = 0;
};

struct Side {
  int ncol = 0;
  int32_t type[TQ_MAX_COLS];
  int64_t rows_per_chunk = 0;
  size_t off[TQ_MAX_COLS];
  std::vector<Holder> parts;
};

class Driver {
 public:
  tq_pagepool* pool;
  tq_budget* budget;
  const tq_ooc_plan& plan;
  hipStream_t copy, compute, spill = nullptr;
  tq_ooc_stats st{};
  int nparts;
  size_t chunk_bytes;

  // workspace
  char* work;
  size_t work_cap;
  size_t fixed_used = 0;
  size_t reserved_fixed = 0;

  // arena of chunks
  char* arena = nullptr;
  int64_t n_chunks = 0;
  std::vector<int64_t> free_chunks;
  std::vector<uint8_t> chunk_busy;  // taken for a contiguous region
  struct Pending {
    hipEvent_t ev;
    std::vector<int64_t> chunks;
  };
  std::deque<Pending> pending;  // chunks to return once an event completes

  // spill store
  std::vector<int32_t> spill_pages;
  int32_t cur_page = -1, cur_sub = 0, subs_per_page = 0;

  Side dim, fact;
  int phase = 1;     // 1: partitioning, 2: joining

  // Adaptive Exchange: 0 while undecided, then TQ_EXCHANGE_PARTITIONED or TQ_EXCHANGE_SINGLE
  int xmode = 0;
  int64_t dim_total = 0, dim_seen = 0;  // dimension rows in all batches / filtered so far
  void* s_table = nullptr;              // single mode: the one join table
  tq_agg s_agg{};
  int pin_lo = 0, pin_hi = -1;  // partitions that must stay resident in pass 2

  // descriptors
  CopyDesc* h_desc = nullptr;
  CopyDesc* d_desc = nullptr;
  int max_desc = 0;
  int64_t* h_counts = nullptr;  // pinned: offsets or counts read back per batch
  int32_t host_run = -1;        // pool pages holding h_desc and h_counts
  int64_t host_run_pages = 0;

  Driver(tq_pagepool* p, tq_budget* b, const tq_ooc_plan& pl, hipStream_t c, hipStream_t k, void* w, size_t wb)
      : pool(p), budget(b), plan(pl), copy(c), compute(k), work(static_cast<char*>(w)), work_cap(wb) {
    nparts = 1 << plan.log2_fanout;
    chunk_bytes = plan.chunk_bytes;
  }

  ~Driver() {
    if (spill) {
      (void)hipStreamSynchronize(spill);
      (void)hipStreamDestroy(spill);
    }
    (void)hipStreamSynchronize(compute);
    (void)hipStreamSynchronize(copy);
    for (auto& q : pending) (void)hipEventDestroy(q.ev);
    if (!spill_pages.empty()) tq_pagepool_free(pool, spill_pages.data(), (int64_t)spill_pages.size());
    if (host_run >= 0) pool_give_run(pool, host_run, host_run_pages);
    if (reserved_fixed) tq_budget_release(budget, reserved_fixed);
    if (chunks_out) tq_budget_release(budget, (size_t)chunks_out * chunk_bytes);
  }

  int64_t chunks_out = 0;  // chunks taken from the arena and not yet returned (each holds a reservation)

  // Carve `bytes` from the front of the workspace, reserved from the budget.
  tq_status carve(size_t bytes, void** out) {
    bytes = align_up(bytes, kAlign);
    if (fixed_used + bytes > work_cap) return fail(TQ_ENOMEM, "workspace too small for the fixed buffers");
    tq_status s = tq_budget_reserve(budget, bytes);
    if (s) return fail(TQ_ENOMEM, "budget cannot hold the fixed buffers (%zu bytes more)", bytes);
    reserved_fixed += bytes;
    *out = work + fixed_used;
    fixed_used += bytes;
    return TQ_OK;
  }

  void setup_side(Side& s, int ncol, const int32_t* types) {
    s.ncol = ncol;
    size_t row = 0;
    for (int c = 0; c < ncol; c++) {
      s.type[c] = types[c];
      row += types[c];
    }
    int64_t R = (int64_t)((chunk_bytes - kAlign * ncol) / row) / 64 * 64;
    s.rows_per_chunk = R;
    size_t off = 0;
    for (int c = 0; c < ncol; c++) {
      s.off[c] = off;
      off = align_up(off + (size_t)R * s.type[c], kAlign);
    }
    s.parts.assign(nparts, Holder());
  }

  char* chunk_ptr(int64_t id) { return arena + (size_t)id * chunk_bytes; }

  // -------------------------------------------------------------- chunks

  tq_status reclaim_one(bool wait) {
    if (pending.empty()) return TQ_ENOMEM;
    Pending& q = pending.front();
    if (wait) TQ_HIP(hipEventSynchronize(q.ev));
    else if (hipEventQuery(q.ev) != hipSuccess) return TQ_ENOMEM;
    (void)hipEventDestroy(q.ev);
    for (int64_t id : q.chunks) {
      free_chunks.push_back(id);
      tq_budget_release(budget, chunk_bytes);
      chunks_out--;
    }
    pending.pop_front();
    return TQ_OK;
  }

  // Returns the chunks `ids` to the arena once the work enqueued so far on `s` is done.
  tq_status retire(std::vector<int64_t> ids, hipStream_t s) {
    if (ids.empty()) return TQ_OK;
    hipEvent_t ev;
    TQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TQ_HIP(hipEventRecord(ev, s));
    pending.push_back(Pending{ev, std::move(ids)});
    return TQ_OK;
  }

  // Pass 1 may spill any resident chunk that no append being assembled writes
  // into, a partly filled tail too: the next append to that partition starts a
  // new chunk, and pass 2 reads every chunk by its own row count.
  bool spillable(int p, const Holder& h, size_t idx) const {
    const ChunkRef& c = h.chunks[idx];
    if (c.dev < 0 || c.pinned) return false;
    if (phase == 1) return true;
    return p < pin_lo || p > pin_hi;
  }

  // Spill one resident chunk of the partition that pass 2 reaches last,
  // preferring full chunks: a partly filled tail that is spilled costs a whole
  // chunk's copy for its few rows, and the partition's next append opens yet
  // another chunk.
  tq_status spill_one(bool* done) {
    *done = false;
    for (int full_only = 1; full_only >= 0; full_only--)
      for (int p = nparts - 1; p >= 0; p--) {
        if (phase == 2 && p <= pin_hi) break;  // earlier partitions are done or pinned
        for (Side* s : {&fact, &dim}) {
          Holder& h = s->parts[p];
          for (size_t i = h.chunks.size(); i-- > 0;) {
            if (!spillable(p, h, i) || (full_only && h.chunks[i].rows < s->rows_per_chunk)) continue;
            TQ_HIP(spill_chunk(h.chunks[i]));
            *done = true;
            return TQ_OK;
          }
        }
      }
    return TQ_OK;
  }

  hipError_t spill_chunk(ChunkRef& c) {
    if (!spill) {
      hipError_t e = hipStreamCreateWithFlags(&spill, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    if (cur_page < 0 || cur_sub == subs_per_page) {
      int32_t id;
      if (tq_pagepool_alloc(pool, 1, &id) != TQ_OK) return hipErrorOutOfMemory;
      spill_pages.push_back(id);
      cur_page = id;
      cur_sub = 0;
    }
    // the spill copy follows everything already enqueued on the compute stream
    // (appends) and on the copy stream (a reload into this chunk)
    for (hipStream_t src : {compute, copy}) {
      hipEvent_t fence;
      hipError_t e = hipEventCreateWithFlags(&fence, hipEventDisableTiming);
      if (e != hipSuccess) return e;
      if ((e = hipEventRecord(fence, src)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(spill, fence, 0)) != hipSuccess) return e;
      (void)hipEventDestroy(fence);
    }
    hipError_t e;
    char* host = static_cast<char*>(tq_pagepool_page(pool, cur_page)) + (size_t)cur_sub * chunk_bytes;
    if ((e = hipMemcpyAsync(host, chunk_ptr(c.dev), chunk_bytes, hipMemcpyDeviceToHost, spill)) != hipSuccess) return e;
    st.bytes_d2h += (int64_t)chunk_bytes;
    st.spilled_chunks++;
    spill_unwaited = true;
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventRecord(ev, spill)) != hipSuccess) return e;
    pending.push_back(Pending{ev, {c.dev}});
    c.dev = -1;
    c.page = cur_page;
    c.sub = cur_sub++;
    return hipSuccess;
  }

  // A free chunk, reserved from the budget, if one is free now (no wait, no spill).
  bool try_take_chunk(int64_t* out) {
    while (reclaim_one(false) == TQ_OK) {
    }
    if (free_chunks.empty() || tq_budget_reserve(budget, chunk_bytes) != TQ_OK) return false;
    *out = free_chunks.back();
    free_chunks.pop_back();
    chunks_out++;
    return true;
  }

  // A free chunk, reserved from the budget; spills when none is available.
  tq_status take_chunk(int64_t* out) {
    for (int guard = 0; guard < (1 << 30); guard++) {
      if (try_take_chunk(out)) return TQ_OK;
      if (!pending.empty()) {
        tq_status s = reclaim_one(true);
        if (s) return s;
        continue;
      }
      // spill several chunks at once, so that their copies to the host run back
      // to back and the wait below is for the first of them only
      bool spilled = false;
      for (int k = 0; k < kSpillBatch; k++) {
        bool one = false;
        tq_status s = spill_one(&one);
        if (s) return s;
        if (!one) break;
        spilled = true;
      }
      if (spilled) continue;
      tq_status s;
      if (appending && !touched.empty()) {
        // every resident chunk is pinned by the append being assembled: launch
        // its copies so far, after which those chunks may be spilled
        if ((s = launch_copies())) return s;
        unpin_touched();
        continue;
      }
      return fail(TQ_ENOMEM, "device budget exhausted and nothing left to spill");
    }
    return fail(TQ_ENOMEM, "chunk allocation did not converge");
  }

  bool spill_unwaited = false;  // spill copies enqueued since the copy stream last waited for them

  // Copies a spilled chunk back into the arena; with `nowait`, only into a
  // chunk that is free now, returning TQ_ENOMEM otherwise.
  tq_status reload(ChunkRef& c, bool nowait = false) {
    if (c.dev >= 0) return TQ_OK;
    int64_t id;
    if (nowait) {
      if (!try_take_chunk(&id)) return TQ_ENOMEM;
    } else {
      tq_status s = take_chunk(&id);
      if (s) return s;
    }
    if (spill_unwaited) {
      // the chunk's spill copy to the host page may still be in flight
      hipEvent_t ev;
      TQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      TQ_HIP(hipEventRecord(ev, spill));
      TQ_HIP(hipStreamWaitEvent(copy, ev, 0));
      TQ_HIP(hipEventDestroy(ev));
      spill_unwaited = false;
    }
    const char* host = static_cast<const char*>(tq_pagepool_page(pool, c.page)) + (size_t)c.sub * chunk_bytes;
    TQ_HIP(hipMemcpyAsync(chunk_ptr(id), host, chunk_bytes, hipMemcpyHostToDevice, copy));
    st.bytes_h2d += (int64_t)chunk_bytes;
    st.reloaded_chunks++;
    c.dev = id;
    return TQ_OK;
  }

  // -------------------------------------------------------------- appends

  std::vector<CopyDesc> descs;
  size_t desc_used = 0;  // descriptor slots of h_desc / d_desc taken since the last sync of `compute`
  bool appending = false;
  Side* app_side = nullptr;
  std::vector<std::pair<int, size_t>> touched;  // (partition, chunk index) pinned by the current append

  void unpin_touched() {
    for (auto& t : touched) app_side->parts[t.first].chunks[t.second].pinned = false;
    touched.clear();
  }

  // Append rows [off[p], off[p+1]) of every partition p from the partitioned
  // columns `src` (side column j at src[j]) to the holders. The caller has
  // synchronised `compute` since the previous append (its offsets were read
  // back), so the descriptor buffers are free.
  tq_status append(Side& s, char* const* src, const int64_t* off) {
    descs.clear();
    desc_used = 0;
    appending = true;
    app_side = &s;
    // a chunk is pinned (not spillable) from the moment a descriptor of this
    // batch targets it until the copy kernel that fills it has been enqueued
    touched.clear();
    tq_status e = TQ_OK;
    for (int p = 0; p < nparts && e == TQ_OK; p++) {
      int64_t at = off[p], left = off[p + 1] - off[p];
      Holder& h = s.parts[p];
      h.rows += left;
      while (left > 0) {
        if (h.chunks.empty() || h.chunks.back().rows == s.rows_per_chunk || h.chunks.back().dev < 0) {
          int64_t id;
          if ((e = take_chunk(&id))) break;
          ChunkRef c;
          c.dev = id;
          h.chunks.push_back(c);
        }
        ChunkRef& c = h.chunks.back();
        if (!c.pinned) {
          c.pinned = true;
          touched.emplace_back(p, h.chunks.size() - 1);
        }
        int64_t m = std::min(left, s.rows_per_chunk - c.rows);
        for (int j = 0; j < s.ncol; j++) {
          int w = s.type[j];
          descs.push_back(CopyDesc{src[j] + (size_t)at * w, chunk_ptr(c.dev) + s.off[j] + (size_t)c.rows * w, m, w, 0});
        }
        c.rows += m;
        at += m;
        left -= m;
      }
    }
    if (e == TQ_OK) e = launch_copies();
    unpin_touched();
    appending = false;
    return e;
  }

  // Enqueues the copies described so far on `compute`, in descriptor slots not
  // used since `compute` was last synchronised (an earlier copy of pinned host
  // descriptors may still be in flight).
  tq_status launch_copies() {
    size_t done = 0;
    while (done < descs.size()) {
      if (desc_used == (size_t)max_desc) {  // every slot is in use: wait until compute has read them
        TQ_HIP(hipStreamSynchronize(compute));
        desc_used = 0;
      }
      const size_t k = std::min({descs.size() - done, (size_t)max_desc - desc_used, (size_t)65535});
      memcpy(h_desc + desc_used, descs.data() + done, k * sizeof(CopyDesc));
      TQ_HIP(hipMemcpyAsync(d_desc + desc_used, h_desc + desc_used, k * sizeof(CopyDesc), hipMemcpyHostToDevice,
                            compute));
      int64_t tiles = 1;
      for (size_t i = done; i < done + k; i++)
        tiles = std::max<int64_t>(tiles, (descs[i].n * descs[i].w + kCopyTile - 1) / kCopyTile);
      const int gx = (int)std::min<int64_t>(tiles, std::max<int64_t>(1, 4096 / (int64_t)k));
      hipLaunchKernelGGL(k_gather_copy, dim3(gx, (unsigned)k), dim3(256), 0, compute, d_desc + desc_used);
      TQ_HIP(hipGetLastError());
      desc_used += k;
      done += k;
    }
    descs.clear();
    return TQ_OK;
  }

  // Waits for `compute` and reads n int64 values from device memory.
  tq_status read_back(const int64_t* d, int64_t n) {
    TQ_HIP(hipMemcpyAsync(h_counts, d, (size_t)n * 8, hipMemcpyDeviceToHost, compute));
    TQ_HIP(hipStreamSynchronize(compute));
    return TQ_OK;
  }

  // -------------------------------------------------------------- passes

  // pass-1 buffers
  int64_t* d_off = nullptr;
  void* d_part_scratch = nullptr;
  size_t part_scratch_bytes = 0;
  char* tmp_a = nullptr;  // dimension filter output: key, payload (int64)
  char* tmp_b = nullptr;  // partition output
  size_t tmp_b_bytes = 0;
  void* fp_scratch = nullptr;
  int64_t* d_count = nullptr;
  int64_t max_dim_rows = 0, max_fact_rows = 0;
  int fact_map[TQ_MAX_COLS];  // fact column -> side column (or -1)
  int fact_src[TQ_MAX_COLS];  // side column -> fact column
  // pass 2: contiguous copy of one partition's probe columns
  char* fg_base = nullptr;
  int64_t fg_rows = 0;
  int fg_ncol = 0;
  int fg_col[TQ_MAX_COLS];     // side column -> index among the copied columns (or -1)
  size_t fg_off[TQ_MAX_COLS];  // side column -> byte offset of its copy

  static tq_status on_dim(void* user, int64_t, const tq_col* cols, int32_t ncol, int64_t nrows, hipStream_t) {
    return static_cast<Driver*>(user)->dim_batch(cols, ncol, nrows);
  }
  static tq_status on_fact(void* user, int64_t, const tq_col* cols, int32_t ncol, int64_t nrows, hipStream_t) {
    return static_cast<Driver*>(user)->fact_batch(cols, ncol, nrows);
  }

  tq_status dim_batch(const tq_col* cols, int32_t ncol, int64_t nrows) {
    if (nrows == 0) return TQ_OK;
    // sigma + pi: keep (key, payload) of the rows that pass, as int64
    tq_expr e[2];
    memset(e, 0, sizeof e);
    e[0].nf = 1;
    e[0].f[0] = tq_factor{plan.dim_key_col, 1, 0};
    e[1].nf = 1;
    e[1].f[0] = tq_factor{plan.dim_payload_col, 1, 0};
    int64_t* outs[2] = {reinterpret_cast<int64_t*>(tmp_a), reinterpret_cast<int64_t*>(tmp_a + align_up((size_t)nrows * 8, kAlign))};
    tq_status s = tq_filter_project(cols, ncol, nrows, plan.dim_preds, plan.dim_np, e, 2, outs, nullptr, d_count, fp_scratch,
                                    tq_filter_project_scratch_bytes(nrows), compute);
    if (s) return s;
    if ((s = read_back(d_count, 1))) return s;
    const int64_t kept = h_counts[0];
    st.dim_rows_kept += kept;
    dim_seen += nrows;
    if (xmode == TQ_EXCHANGE_SINGLE) {
      // one table: the kept rows need no partitioning, they all go to the first holder
      for (int q = 0; q <= nparts; q++) h_counts[q] = q == 0 ? 0 : kept;
      char* src[2] = {reinterpret_cast<char*>(outs[0]), reinterpret_cast<char*>(outs[1])};
      return append(dim, src, h_counts);
    }
    char* out_key = tmp_b;
    char* out_pay = tmp_b + align_up((size_t)kept * 8, kAlign);
    tq_col pay = {outs[1], TQ_I64};
    void* outp[1] = {out_pay};
    s = tq_hash_partition(outs[0], &pay, 1, kept, plan.log2_fanout, 0, reinterpret_cast<int64_t*>(out_key), outp, d_off,
                          d_part_scratch, part_scratch_bytes, compute);
    if (s) return s;
    if ((s = read_back(d_off, nparts + 1))) return s;
    char* src[2] = {out_key, out_pay};
    if ((s = append(dim, src, h_counts))) return s;
    if (xmode == 0 && dim_seen * 8 >= dim_total) decide();
    return TQ_OK;
  }

  // Adaptive Exchange, first phase (Section 3.2): the kept fraction of the
  // dimension rows filtered so far, applied to all of them, estimates the
  // filtered dimension; one table is chosen when that estimate, with a quarter
  // more for its error, fits the arena beside the holders of its rows. On one
  // GPU the host link bounds this path, so the budget is the only criterion:
  // a single table saves the fact side's exchange whatever the table's size
  // relative to the caches.
  void decide() {
    const int64_t est = dim_seen > 0 ? (int64_t)((double)st.dim_rows_kept * (double)dim_total / (double)dim_seen + 0.5) : 0;
    st.est_dim_rows = est;
    st.est_from_rows = dim_seen;
    const int64_t rows = est + est / 4 + 1024;
    const int64_t holder_chunks = (rows + dim.rows_per_chunk - 1) / dim.rows_per_chunk + nparts;
    const size_t region = single_region_bytes(rows);
    const int64_t region_chunks = (int64_t)((region + chunk_bytes - 1) / chunk_bytes);
    xmode = holder_chunks + region_chunks <= n_chunks ? TQ_EXCHANGE_SINGLE : TQ_EXCHANGE_PARTITIONED;
  }

  static size_t gather_bytes_for(int64_t rows) { return 2 * align_up((size_t)std::max<int64_t>(rows, 1) * 8, kAlign); }
  size_t single_region_bytes(int64_t rows) const {
    return gather_bytes_for(rows) + tq_join_table_bytes(std::max<int64_t>(rows, 1), plan.load_factor);
  }

  // Single mode: gathers every kept dimension row into one contiguous copy and
  // builds one table over it, then releases the holders. *fits is false (and
  // nothing is enqueued) when the budget cannot hold the table and the copy
  // beside the holders, or when holders were spilled.
  tq_status single_table(bool* fits) {
    *fits = false;
    for (Holder& h : dim.parts)
      for (ChunkRef& c : h.chunks)
        if (c.dev < 0) return TQ_OK;
    const int64_t n = st.dim_rows_kept;
    const size_t table_bytes = tq_join_table_bytes(std::max<int64_t>(n, 1), plan.load_factor);
    char* region;
    tq_status s = take_region(single_region_bytes(n), &region, false);
    if (s == TQ_ENOMEM) return TQ_OK;
    if (s) return s;
    *fits = true;
    int64_t* g_key = reinterpret_cast<int64_t*>(region);
    int64_t* g_pay = reinterpret_cast<int64_t*>(region + align_up((size_t)std::max<int64_t>(n, 1) * 8, kAlign));
    s_table = region + gather_bytes_for(n);
    if ((s = tq_join_table_init(s_table, table_bytes, compute))) return s;
    descs.clear();
    int64_t at = 0;
    for (Holder& h : dim.parts)
      for (ChunkRef& c : h.chunks) {
        descs.push_back(CopyDesc{chunk_ptr(c.dev) + dim.off[0], g_key + at, c.rows, 8, 0});
        descs.push_back(CopyDesc{chunk_ptr(c.dev) + dim.off[1], g_pay + at, c.rows, 8, 0});
        at += c.rows;
      }
    if ((s = launch_copies())) return s;
    tq_col pc = {g_pay, TQ_I64};
    if ((s = tq_join_build(s_table, table_bytes, g_key, pc, at, nullptr, 0, nullptr, 0, plan.load_factor, 0,
                           plan.join_flags, compute)))
      return s;
    return release_dim();
  }

  // Drops the dimension's holders: resident chunks return to the arena once
  // `compute` has passed this point; spilled ones keep their pool pages until
  // the call ends.
  tq_status release_dim() {
    std::vector<int64_t> ids;
    for (Holder& h : dim.parts)
      for (ChunkRef& c : h.chunks)
        if (c.dev >= 0) ids.push_back(c.dev);
    dim.parts.assign(nparts, Holder());
    return retire(std::move(ids), compute);
  }

  tq_status fact_batch(const tq_col* cols, int32_t ncol, int64_t nrows) {
    if (nrows == 0) return TQ_OK;
    st.fact_rows += nrows;
    if (xmode == TQ_EXCHANGE_SINGLE)  // no exchange: probe the staged batch where it lies
      return tq_join_probe(s_table, static_cast<const int64_t*>(cols[plan.fact_key_col].data), nrows, cols, ncol, nullptr,
                           0, nullptr, nullptr, 0, nullptr, &s_agg, compute);
    char* src[TQ_MAX_COLS];
    tq_col pay[TQ_MAX_COLS] = {};
    void* outp[TQ_MAX_COLS];
    size_t off = 0;
    for (int j = 0; j < fact.ncol; j++) {
      src[j] = tmp_b + off;
      off = align_up(off + (size_t)nrows * fact.type[j], kAlign);
      if (j > 0) {
        pay[j - 1] = cols[fact_src[j]];
        outp[j - 1] = src[j];
      }
    }
    (void)ncol;
    tq_status s = tq_hash_partition(static_cast<const int64_t*>(cols[plan.fact_key_col].data), pay, fact.ncol - 1, nrows,
                                    plan.log2_fanout, 0, reinterpret_cast<int64_t*>(src[0]), outp, d_off, d_part_scratch,
                                    part_scratch_bytes, compute);
    if (s) return s;
    if ((s = read_back(d_off, nparts + 1))) return s;
    return append(fact, src, h_counts);
  }

  tq_status run(const tq_batch* dimb, int64_t nd, const tq_batch* factb, int64_t nf, void* d_state) {
    auto t0 = std::chrono::steady_clock::now();
    // ---- sides
    int32_t dim_types[2] = {TQ_I64, TQ_I64};
    setup_side(dim, 2, dim_types);
    int32_t ft[TQ_MAX_COLS];
    int nk = 0;
    const tq_batch& f0 = factb[0];
    for (int c = 0; c < TQ_MAX_COLS; c++) fact_map[c] = -1;
    ft[nk] = f0.col_type[plan.fact_key_col];
    fact_map[plan.fact_key_col] = nk;
    fact_src[nk++] = plan.fact_key_col;
    for (int c = 0; c < f0.ncol; c++)
      if (((plan.fact_keep_mask >> c) & 1) && c != plan.fact_key_col) {
        ft[nk] = f0.col_type[c];
        fact_map[c] = nk;
        fact_src[nk++] = c;
      }
    setup_side(fact, nk, ft);
    if (dim.rows_per_chunk < 64 || fact.rows_per_chunk < 64) return fail(TQ_EINVAL, "chunk_bytes too small for a row");
    subs_per_page = (int32_t)(tq_pagepool_page_bytes(pool) / chunk_bytes);

    // ---- fixed buffers
    size_t max_batch = 0;
    for (int64_t i = 0; i < nd; i++) {
      max_batch = std::max(max_batch, (size_t)dimb[i].npages * tq_pagepool_page_bytes(pool));
      max_dim_rows = std::max(max_dim_rows, dimb[i].nrows);
    }
    for (int64_t i = 0; i < nf; i++) {
      max_batch = std::max(max_batch, (size_t)factb[i].npages * tq_pagepool_page_bytes(pool));
      max_fact_rows = std::max(max_fact_rows, factb[i].nrows);
    }
    const int64_t max_rows = std::max(max_dim_rows, max_fact_rows);
    void* staging;
    tq_status s;
    if ((s = carve(max_batch * plan.nslots, &staging))) return s;
    void* p;
    if ((s = carve(2 * align_up((size_t)max_dim_rows * 8, kAlign), &p))) return s;
    tmp_a = static_cast<char*>(p);
    size_t fact_row = 0;
    for (int j = 0; j < fact.ncol; j++) fact_row += fact.type[j];
    tmp_b_bytes = std::max((size_t)max_fact_rows * fact_row + kAlign * fact.ncol, 2 * align_up((size_t)max_dim_rows * 8, kAlign));
    if ((s = carve(tmp_b_bytes, &p))) return s;
    tmp_b = static_cast<char*>(p);
    part_scratch_bytes = tq_hash_partition_scratch_bytes(max_rows, plan.log2_fanout);
    if ((s = carve(part_scratch_bytes, &d_part_scratch))) return s;
    if ((s = carve((size_t)(nparts + 1) * 8, &p))) return s;
    d_off = static_cast<int64_t*>(p);
    if ((s = carve(tq_filter_project_scratch_bytes(max_dim_rows) + 64, &fp_scratch))) return s;
    if ((s = carve(64, &p))) return s;
    d_count = static_cast<int64_t*>(p);
    max_desc = nparts * (TQ_MAX_COLS + 1) * 4 + 64;
    if ((s = carve((size_t)max_desc * sizeof(CopyDesc), &p))) return s;
    d_desc = static_cast<CopyDesc*>(p);
    {
      // host staging from consecutive pool pages (pinned once with the pool), not pinned per call
      const size_t desc_bytes = align_up((size_t)max_desc * sizeof(CopyDesc), kAlign);
      const size_t page = tq_pagepool_page_bytes(pool);
      const int64_t np = (int64_t)((desc_bytes + (size_t)(nparts + 8) * 8 + page - 1) / page);
      if ((s = pool_take_run(pool, np, &host_run)))
        return fail(TQ_ENOMEM, "the page pool has no %lld consecutive free pages for the copy descriptors", (long long)np);
      host_run_pages = np;
      char* hb = static_cast<char*>(tq_pagepool_page(pool, host_run));
      h_desc = reinterpret_cast<CopyDesc*>(hb);
      h_counts = reinterpret_cast<int64_t*>(hb + desc_bytes);
    }

    // ---- arena: the rest of the workspace, within the budget
    size_t cap_left = tq_budget_cap(budget) > tq_budget_used(budget) ? tq_budget_cap(budget) - tq_budget_used(budget) : 0;
    size_t room = std::min(work_cap - align_up(fixed_used, chunk_bytes), cap_left);
    arena = work + align_up(fixed_used, chunk_bytes);
    n_chunks = (int64_t)(room / chunk_bytes);
    if (n_chunks < 4) return fail(TQ_ENOMEM, "budget leaves room for %lld chunks", (long long)n_chunks);
    for (int64_t i = n_chunks - 1; i >= 0; i--) free_chunks.push_back(i);

    // ---- pass 1, dimension side
    phase = 1;
    for (int64_t i = 0; i < nd; i++) dim_total += dimb[i].nrows;
    xmode = plan.exchange;  // TQ_EXCHANGE_AUTO (0) decides after the first batches
    if ((s = stream_dim(dimb, nd, staging, max_batch))) return s;
    if (xmode == 0) decide();
    if (xmode == TQ_EXCHANGE_SINGLE) {
      bool fits = false;
      if ((s = single_table(&fits))) return s;
      if (!fits) {
        if (plan.exchange == TQ_EXCHANGE_SINGLE)
          return fail(TQ_ENOMEM, "one table over %lld dimension rows does not fit the budget", (long long)st.dim_rows_kept);
        // the estimate was too low: stream the dimension side again, partitioned
        if ((s = release_dim())) return s;
        xmode = TQ_EXCHANGE_PARTITIONED;
        st.dim_restreams++;
        st.dim_rows_kept = 0;
        dim_seen = 0;
        if ((s = stream_dim(dimb, nd, staging, max_batch))) return s;
      }
    }
    st.exchange = xmode;
    if (xmode == TQ_EXCHANGE_SINGLE) {
      // ---- the fact side, probing the one table batch by batch
      TQ_HIP(hipStreamSynchronize(compute));
      auto t1 = std::chrono::steady_clock::now();
      s_agg = tq_agg{d_state, plan.domain, plan.sums, plan.nsum};
      if ((s = tq_pagepool_stream(pool, factb, nf, staging, max_batch * plan.nslots, plan.nslots, on_fact, this, copy,
                                  compute)))
        return s;
      for (int64_t i = 0; i < nf; i++) st.bytes_h2d += batch_bytes(factb[i]);
      TQ_HIP(hipStreamSynchronize(compute));
      return finish_stats(t0, t1, std::chrono::steady_clock::now());
    }

    // ---- pass 2 buffers, sized by the largest dimension partition and taken
    // now, while the arena is still mostly free: the gathered partition and its table
    int64_t max_part = 1;
    for (int q = 0; q < nparts; q++) max_part = std::max(max_part, dim.parts[q].rows);
    size_t gather_bytes = 2 * align_up((size_t)max_part * 8, kAlign);
    size_t table_bytes = tq_join_table_bytes(max_part, plan.load_factor);
    // a contiguous copy of one partition's probe columns (its key and the
    // columns the sums read), so that a partition is probed with one launch;
    // sized for 1.3x an even share of the fact rows (a larger partition is
    // probed chunk by chunk instead)
    int64_t fact_total = 0;
    for (int64_t i = 0; i < nf; i++) fact_total += factb[i].nrows;
    fg_rows = fact_total / nparts * 13 / 10 + fact.rows_per_chunk;
    fg_ncol = 0;
    size_t fg_bytes = 0;
    for (int j = 0; j < fact.ncol; j++) {
      const int fc = fact_src[j];
      bool used = fc == plan.fact_key_col;
      for (int e = 0; e < plan.nsum; e++)
        for (int f = 0; f < plan.sums[e].nf; f++) used = used || plan.sums[e].f[f].col == fc;
      fg_col[j] = -1;
      if (used) {
        fg_col[j] = fg_ncol++;
        fg_off[j] = fg_bytes;
        fg_bytes = align_up(fg_bytes + (size_t)fg_rows * fact.type[j], kAlign);
      }
    }
    if (fg_bytes > tq_budget_cap(budget) / 8) fg_rows = 0;  // too large a share of the budget: probe by chunks
    char* region;
    if (fg_rows > 0) {
      s = take_region(gather_bytes + table_bytes + fg_bytes, &region);
      if (s == TQ_ENOMEM) fg_rows = 0;
      else if (s) return s;
    }
    if (fg_rows == 0 && (s = take_region(gather_bytes + table_bytes, &region))) return s;
    fg_base = region + gather_bytes + table_bytes;
    int64_t* g_key = reinterpret_cast<int64_t*>(region);
    int64_t* g_pay = reinterpret_cast<int64_t*>(region + align_up((size_t)max_part * 8, kAlign));
    void* table = region + gather_bytes;
    if ((s = tq_join_table_init(table, table_bytes, compute))) return s;
    phase = 1;

    // ---- pass 1, fact side
    if ((s = tq_pagepool_stream(pool, factb, nf, staging, max_batch * plan.nslots, plan.nslots, on_fact, this, copy, compute)))
      return s;
    for (int64_t i = 0; i < nf; i++) st.bytes_h2d += batch_bytes(factb[i]);
    TQ_HIP(hipStreamSynchronize(compute));
    auto t1 = std::chrono::steady_clock::now();

    // ---- pass 2
    phase = 2;
    tq_agg agg{d_state, plan.domain, plan.sums, plan.nsum};
    hipEvent_t loaded;
    TQ_HIP(hipEventCreateWithFlags(&loaded, hipEventDisableTiming));
    int ahead = 0;
    for (int q = 0; q < nparts; q++) {
      pin_lo = q;
      pin_hi = q;  // chunks prefetched for later partitions may be spilled again if q needs the room
      if ((s = make_resident(q))) return s;
      TQ_HIP(hipEventRecord(loaded, copy));
      TQ_HIP(hipStreamWaitEvent(compute, loaded, 0));
      // gather the partition's dimension rows (launch_copies waits for compute
      // only when every descriptor slot has been used since it last did)
      descs.clear();
      int64_t at = 0;
      for (ChunkRef& c : dim.parts[q].chunks) {
        descs.push_back(CopyDesc{chunk_ptr(c.dev) + dim.off[0], g_key + at, c.rows, 8, 0});
        descs.push_back(CopyDesc{chunk_ptr(c.dev) + dim.off[1], g_pay + at, c.rows, 8, 0});
        at += c.rows;
      }
      // and its probe columns, when they fit the contiguous copy
      const bool whole = fact.parts[q].rows <= fg_rows;
      int64_t fat = 0;
      if (whole) {
        for (ChunkRef& c : fact.parts[q].chunks) {
          for (int j = 0; j < fact.ncol; j++)
            if (fg_col[j] >= 0)
              descs.push_back(CopyDesc{chunk_ptr(c.dev) + fact.off[j], fg_base + fg_off[j] + (size_t)fat * fact.type[j],
                                       c.rows, fact.type[j], 0});
          fat += c.rows;
        }
      }
      if ((s = launch_copies())) return s;
      tq_col pc = {g_pay, TQ_I64};
      if ((s = tq_join_build(table, table_bytes, g_key, pc, at, nullptr, 0, nullptr, 0, plan.load_factor,
                             plan.log2_fanout, plan.join_flags, compute)))
        return s;
      if (whole && fat > 0) {
        tq_col cols[TQ_MAX_COLS] = {};
        int ncols = 0;
        const int jk = fact_map[plan.fact_key_col];
        for (int fc = 0; fc < TQ_MAX_COLS; fc++) {
          int j = fact_map[fc];
          if (j >= 0 && fg_col[j] >= 0) {
            ncols = fc + 1;
            cols[fc].data = fg_base + fg_off[j];
            cols[fc].type = fact.type[j];
          } else {  // a column no sum reads: any valid pointer (the plan never loads it)
            cols[fc].data = fg_base + fg_off[jk];
            cols[fc].type = fact.type[jk];
          }
        }
        if ((s = tq_join_probe(table, reinterpret_cast<const int64_t*>(fg_base + fg_off[jk]), fat, cols, ncols, nullptr, 0,
                               nullptr, nullptr, 0, nullptr, &agg, compute)))
          return s;
      }
      for (ChunkRef& c : fact.parts[q].chunks) {
        if (whole) break;
        tq_col cols[TQ_MAX_COLS] = {};
        int ncols = 0;
        for (int fc = 0; fc < TQ_MAX_COLS; fc++) {
          int j = fact_map[fc];
          if (j >= 0) ncols = fc + 1;
          cols[fc].data = chunk_ptr(c.dev) + (j >= 0 ? fact.off[j] : fact.off[0]);
          cols[fc].type = j >= 0 ? fact.type[j] : fact.type[0];
        }
        if ((s = tq_join_probe(table, reinterpret_cast<const int64_t*>(chunk_ptr(c.dev) + fact.off[0]), c.rows, cols, ncols,
                               nullptr, 0, nullptr, nullptr, 0, nullptr, &agg, compute)))
          return s;
      }
      // partition q is done once the compute stream passes this point
      std::vector<int64_t> done;
      for (Side* sd : {&dim, &fact})
        for (ChunkRef& c : sd->parts[q].chunks) {
          done.push_back(c.dev);
          c.dev = -1;
        }
      if ((s = retire(std::move(done), compute))) return s;
      // reload the next partitions ahead of use, overlapping q's compute; what
      // the budget cannot hold now is loaded when its partition is reached
      pin_lo = q;
      int a = 1;
      for (; a <= kPrefetchParts && q + a < nparts; a++) {
        pin_hi = q + a;
        s = make_resident(q + a);
        if (s == TQ_ENOMEM) {
          s = TQ_OK;
          break;
        }
        if (s) return s;
      }
      // and, in partition order, as many later ones as the chunks free now
      // hold, so that the copy engine is busy from the start of the pass
      if (a > kPrefetchParts) {
        for (int r = std::max(q + a, ahead); r < nparts; r++) {
          s = make_resident(r, true);
          if (s == TQ_ENOMEM) {
            s = TQ_OK;
            break;
          }
          if (s) return s;
          ahead = r + 1;  // partitions before `ahead` are resident
        }
      }
    }
    (void)hipEventDestroy(loaded);
    TQ_HIP(hipStreamSynchronize(compute));
    return finish_stats(t0, t1, std::chrono::steady_clock::now());
  }

  tq_status stream_dim(const tq_batch* dimb, int64_t nd, void* staging, size_t max_batch) {
    tq_status s = tq_pagepool_stream(pool, dimb, nd, staging, max_batch * plan.nslots, plan.nslots, on_dim, this, copy,
                                     compute);
    if (s) return s;
    for (int64_t i = 0; i < nd; i++) st.bytes_h2d += batch_bytes(dimb[i]);
    return TQ_OK;
  }

  using Clock = std::chrono::steady_clock;
  tq_status finish_stats(Clock::time_point t0, Clock::time_point t1, Clock::time_point t2) {
    st.ms_pass1 = std::chrono::duration<double, std::milli>(t1 - t0).count();
    st.ms_pass2 = std::chrono::duration<double, std::milli>(t2 - t1).count();
    st.ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
    st.peak_budget_bytes = (int64_t)tq_budget_peak(budget);
    return TQ_OK;
  }

  static int64_t batch_bytes(const tq_batch& b) {
    int64_t end = 0;
    for (int c = 0; c < b.ncol; c++) end = std::max(end, b.col_offset[c] + b.nrows * b.col_type[c]);
    return end;
  }

  tq_status make_resident(int q, bool nowait = false) {
    for (Side* sd : {&dim, &fact})
      for (ChunkRef& c : sd->parts[q].chunks) {
        tq_status s = reload(c, nowait);
        if (s) return s;
      }
    return TQ_OK;
  }

  // A contiguous run of arena chunks (reserved from the budget) for pass-2 buffers.
  // Without `may_spill`, only the arena's free chunks are searched (after every
  // pending release has completed) and TQ_ENOMEM is returned quietly.
  tq_status take_region(size_t bytes, char** out, bool may_spill = true) {
    int64_t need = (int64_t)((bytes + chunk_bytes - 1) / chunk_bytes);
    for (int attempt = 0; attempt < 4; attempt++) {
      while (reclaim_one(!may_spill) == TQ_OK) {
      }
      std::vector<uint8_t> is_free((size_t)n_chunks, 0);
      for (int64_t id : free_chunks) is_free[(size_t)id] = 1;
      int64_t run = 0;
      for (int64_t id = n_chunks - 1; id >= 0; id--) {
        run = is_free[(size_t)id] ? run + 1 : 0;
        if (run == need) {
          if (tq_budget_reserve(budget, (size_t)need * chunk_bytes) != TQ_OK) {
            run = 0;
            break;
          }
          std::vector<int64_t> rest;
          for (int64_t f : free_chunks)
            if (f < id || f >= id + need) rest.push_back(f);
          free_chunks.swap(rest);
          reserved_fixed += (size_t)need * chunk_bytes;
          *out = chunk_ptr(id);
          return TQ_OK;
        }
      }
      if (!may_spill) return TQ_ENOMEM;
      // make room: spill pass-1 data of the last partitions, then retry
      phase = 2;
      pin_lo = 0;
      pin_hi = -1;
      for (int64_t k = 0; k < need; k++) {
        bool spilled = false;
        tq_status s = spill_one(&spilled);
        if (s || !spilled) break;
      }
      while (!pending.empty())
        if (reclaim_one(true)) break;
    }
    return fail(TQ_ENOMEM, "no contiguous %zu bytes for the pass-2 buffers", bytes);
  }
};

}  // namespace
}  // namespace tq

extern "C" tq_status tq_ooc_join_agg(tq_pagepool* pool, const tq_batch* dim, int64_t nd, const tq_batch* fact, int64_t nf,
                                     const tq_ooc_plan* plan, tq_budget* budget, void* d_work, size_t work_bytes,
                                     void* d_state, tq_ooc_stats* stats, hipStream_t copy, hipStream_t compute) {
  using tq::fail;
  if (!pool || !plan || !budget || !d_work || !d_state) return fail(TQ_EINVAL, "NULL argument");
  if (nd < 0 || nf < 1 || (nd > 0 && !dim) || !fact) return fail(TQ_EINVAL, "batch lists");
  if (plan->log2_fanout < 0 || plan->log2_fanout > 10) return fail(TQ_EINVAL, "log2_fanout outside [0, 10]");
  if (plan->join_flags & ~TQ_UNIQUE_KEYS) return fail(TQ_EINVAL, "join_flags: only TQ_UNIQUE_KEYS applies here");
  if (plan->nslots < 2 || plan->nslots > 8) return fail(TQ_EINVAL, "nslots outside [2, 8]");
  if (plan->exchange < TQ_EXCHANGE_AUTO || plan->exchange > TQ_EXCHANGE_SINGLE) return fail(TQ_EINVAL, "exchange mode");
  size_t pb = tq_pagepool_page_bytes(pool);
  if (plan->chunk_bytes < 65536 || plan->chunk_bytes % 256 || pb % plan->chunk_bytes)
    return fail(TQ_EINVAL, "chunk_bytes must be a multiple of 256, at least 64 KiB, and divide the page size");
  for (int64_t i = 0; i < nf; i++) {
    const tq_batch& b = fact[i];
    if (b.ncol != fact[0].ncol || b.ncol > TQ_MAX_COLS) return fail(TQ_EINVAL, "fact batches differ in columns");
    for (int c = 0; c < b.ncol; c++)
      if (b.col_type[c] != fact[0].col_type[c]) return fail(TQ_EINVAL, "fact batches differ in column types");
  }
  const tq_batch& f0 = fact[0];
  if (plan->fact_key_col < 0 || plan->fact_key_col >= f0.ncol || f0.col_type[plan->fact_key_col] != TQ_I64)
    return fail(TQ_EINVAL, "fact key column");
  if (!((plan->fact_keep_mask >> plan->fact_key_col) & 1)) return fail(TQ_EINVAL, "fact_keep_mask must include the key");
  for (int j = 0; j < plan->nsum; j++)
    for (int f = 0; f < plan->sums[j].nf; f++) {
      int c = plan->sums[j].f[f].col;
      if (c >= 0 && (c >= f0.ncol || !((plan->fact_keep_mask >> c) & 1)))
        return fail(TQ_EINVAL, "sum %d reads fact column %d, which is not kept", j, c);
    }
  for (int64_t i = 0; i < nd; i++) {
    const tq_batch& b = dim[i];
    if (plan->dim_key_col < 0 || plan->dim_key_col >= b.ncol || b.col_type[plan->dim_key_col] != TQ_I64 ||
        plan->dim_payload_col < 0 || plan->dim_payload_col >= b.ncol)
      return fail(TQ_EINVAL, "dimension key/payload column");
  }
  tq::Driver d(pool, budget, *plan, copy, compute, d_work, work_bytes);
  tq_status s = d.run(dim, nd, fact, nf, d_state);
  if (stats) *stats = d.st;
  return s;
}
