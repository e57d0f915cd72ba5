// The serving loop: admission by device-memory budget (join tables reserved
// from a history of the kept fraction, with a retry when that proves too
// small), worker threads with their own streams, per-request latency stamps.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace tq {
namespace {

using Clock = std::chrono::steady_clock;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// First-fit allocator over the device arena (offsets only; host side).
class Arena {
 public:
  explicit Arena(size_t bytes) { free_[0] = bytes; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t left = it->second - bytes;
        size_t next = it->first + bytes;
        free_.erase(it);
        if (left) free_[next] = left;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = al(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Plan {  // device memory of one request, as offsets into its region
  size_t state, table, keys, count, sums, avg, ngroups, staging, scratch, total;
  size_t state_bytes, table_bytes, staging_bytes;
  int64_t domain;
  int nsum;
};

tq_col window(const tq_col& c, int64_t first) {
  tq_col w = c;
  w.data = static_cast<const char*>(c.data) + (size_t)first * c.type;
  return w;
}

struct Server {
  const tq_serve_tables& T;
  const tq_request* reqs;
  int64_t n;
  tq_budget* budget;
  char* arena_base;
  Arena arena;
  int64_t max_groups;
  int64_t *h_keys, *h_count, *h_sums;
  double* h_avg;
  tq_request_result* res;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;
  struct Slot {
    int64_t job = -1, rows = 0;
    size_t off = 0, bytes = 0;
    int split = 0;  // the join runs as 2^split hash partitions (0: whole)
    bool busy = false;
  };
  static constexpr int kMaxSplitBits = 8;
  std::vector<Slot> slots;
  bool shutdown = false;
  int64_t completed = 0;

  Server(const tq_serve_tables& t, const tq_request* r, int64_t nr, tq_budget* b, void* d_arena, size_t arena_bytes,
         int64_t mg, int64_t* k, int64_t* c, int64_t* s, double* a, tq_request_result* out)
      : T(t), reqs(r), n(nr), budget(b), arena_base(static_cast<char*>(d_arena)), arena(arena_bytes), max_groups(mg),
        h_keys(k), h_count(c), h_sums(s), h_avg(a), res(out) {}

  double now_s() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // Memory-use history (Section 3.3.2): the kept fraction of the dimension
  // window of the last kHist completed joins of each shape.
  static constexpr int kHist = 16;
  struct History {
    double f[kHist];
    int n = 0, at = 0;
    void add(double x) {
      f[at] = x;
      at = (at + 1) % kHist;
      n = std::min(n + 1, kHist);
    }
  } hist[3];
  std::vector<int64_t> exact;  // per request: kept rows recorded by a build that did not fit, else -1
  std::vector<int32_t> split_min;  // per request: split bits at least (raised when a partition did not fit)
  std::vector<int32_t> retries;
  std::vector<double> first_start;  // per request: when its first run started (-1 before)
  std::deque<int64_t> again;   // requests to run again, ahead of new arrivals

  // The rows a request's table is sized for (called with `mu` held).
  int64_t table_rows(int64_t i) const {
    const tq_request& q = reqs[i];
    if (q.shape == 0) return 0;
    if (exact[(size_t)i] >= 0) return exact[(size_t)i];
    const History& h = hist[q.shape];
    if (!T.estimate || h.n == 0) return q.n_dim;
    double fmax = 0;
    for (int j = 0; j < h.n; j++) fmax = std::max(fmax, h.f[j]);
    const double est = (double)q.n_dim * fmax * 1.25 + 1024.0;
    return est >= (double)q.n_dim ? q.n_dim : (int64_t)est;
  }

  // Table rows of one of 2^b partitions of `rows` kept rows: its share, plus a
  // quarter and 1024 rows for the spread of the hash.
  static int64_t part_rows(int64_t rows, int b) {
    if (b == 0) return rows;
    const double share = (double)rows / (double)(1 << b);
    return std::min<int64_t>(rows, (int64_t)(share * 1.25) + 1024);
  }

  Plan plan_of(const tq_request& q, int64_t table_rows) const {
    Plan p{};
    p.domain = q.shape == 0 ? T.fg_domain : T.join_domain;
    p.nsum = q.shape == 0 ? T.fg_nsum : T.join_nsum;
    p.state_bytes = tq_groupby_state_bytes(p.domain, p.nsum);
    p.table_bytes = q.shape == 0 ? 0 : tq_join_table_bytes(table_rows, T.load_factor);
    size_t staging = 0;
    if (q.shape == 2) {
      size_t mx = 0;
      for (int64_t b = q.fact_first; b < q.fact_first + q.n_fact; b++)
        mx = std::max(mx, (size_t)T.fact_batches[b].npages * tq_pagepool_page_bytes(T.pool));
      staging = mx * (size_t)T.nslots;
    }
    p.staging_bytes = staging;
    size_t o = 0;
    auto take = [&](size_t b) {
      size_t at = o;
      o += al(std::max<size_t>(b, 8));
      return at;
    };
    p.state = take(p.state_bytes);
    p.table = take(p.table_bytes);
    p.keys = take(p.domain * 8);
    p.count = take(p.domain * 8);
    p.sums = take(p.domain * p.nsum * 8);
    p.avg = take(p.domain * p.nsum * 8);
    p.ngroups = take(8);
    p.staging = take(staging);
    p.scratch = take(64);
    p.total = o;
    return p;
  }

  struct ProbeCtx {
    const Server* s;
    void* table;
    tq_agg agg;
  };

  static tq_status on_batch(void* user, int64_t, const tq_col* cols, int32_t, int64_t nrows, hipStream_t compute) {
    auto* c = static_cast<ProbeCtx*>(user);
    const tq_serve_tables& T = c->s->T;
    tq_col fc[4] = {};
    for (int j = 0; j < T.fact_ncol; j++) fc[j] = cols[T.fact_map[j]];
    return tq_join_probe(c->table, static_cast<const int64_t*>(fc[0].data), nrows, fc, T.fact_ncol, nullptr, 0, nullptr,
                         nullptr, 0, nullptr, &c->agg, compute);
  }

  // Runs request idx in the region at `base` (planned for `rows` table rows).
  // *kept gets the rows its dimension window kept (-1 for shape 0). Returns
  // TQ_EFULL, with no result written, when the table was too small for them.
  tq_status execute(const tq_request& q, char* base, int64_t rows, int split, hipStream_t compute, hipStream_t copy,
                    int64_t idx, int64_t* kept) {
    *kept = -1;
    Plan p = plan_of(q, rows);
    void* state = base + p.state;
    int64_t* keys = reinterpret_cast<int64_t*>(base + p.keys);
    int64_t* count = reinterpret_cast<int64_t*>(base + p.count);
    int64_t* sums = reinterpret_cast<int64_t*>(base + p.sums);
    double* avg = reinterpret_cast<double*>(base + p.avg);
    int64_t* ng = reinterpret_cast<int64_t*>(base + p.ngroups);
    tq_status s;
    if ((s = tq_groupby_init(state, p.state_bytes, p.domain, p.nsum, compute))) return s;
    if (q.shape == 0) {
      tq_col w[TQ_MAX_COLS] = {};
      for (int c = 0; c < T.fg_ncol; c++) w[c] = window(T.fg_cols[c], q.fact_first);
      if ((s = tq_groupby_agg(state, p.domain, w, T.fg_ncol, q.n_fact, T.fg_preds, T.fg_np, &T.fg_key, T.fg_sums,
                              T.fg_nsum, compute)))
        return s;
    } else {
      void* table = base + p.table;
      tq_col dw[4] = {};
      for (int c = 0; c < T.dim_ncol; c++) dw[c] = window(T.dim_cols[c], q.dim_first);
      if ((s = tq_join_table_init(table, p.table_bytes, compute))) return s;
      tq_agg agg{state, p.domain, T.join_sums, T.join_nsum};
      int64_t kept_all = 0;
      // whole, or one hash partition after another into the one state (a split)
      for (int part = 0; part < (1 << split); part++) {
        const uint32_t flags = TQ_UNIQUE_KEYS | (split ? TQ_SELECT_PARTITION | TQ_PARTITION(part) : 0u);
        if ((s = tq_join_build(table, p.table_bytes, static_cast<const int64_t*>(dw[0].data), dw[1], q.n_dim, dw,
                               T.dim_ncol, T.dim_preds, T.dim_np, T.load_factor, split, flags, compute)))
          return s;
        if (split) {  // each partition's build is checked before its probe
          int64_t k = 0;
          if ((s = tq_join_table_rows(table, &k, compute))) return s;
          kept_all += k;
          const tq_status t = tq_check(table, compute);
          if (t == TQ_EFULL) {
            *kept = k;
            return t;  // this partition's rows do not fit its table: run again with more partitions
          }
          if (t) return t;
        }
        if (q.shape == 1) {
          tq_col fw[4] = {};
          for (int c = 0; c < T.fact_ncol; c++) fw[c] = window(T.fact_cols[c], q.fact_first);
          if ((s = tq_join_probe(table, static_cast<const int64_t*>(fw[0].data), q.n_fact, fw, T.fact_ncol, nullptr, 0,
                                 nullptr, nullptr, 0, nullptr, &agg, compute)))
            return s;
        } else {
          ProbeCtx ctx{this, table, agg};
          if ((s = tq_pagepool_stream(T.pool, T.fact_batches + q.fact_first, q.n_fact, base + p.staging,
                                      p.staging_bytes, T.nslots, on_batch, &ctx, copy, compute)))
            return s;
        }
      }
      if (split) *kept = kept_all;
    }
    if ((s = tq_groupby_finalize(state, keys, count, sums, avg, ng, compute))) return s;
    if (q.shape != 0 && !split) {
      if ((s = tq_join_table_rows(base + p.table, kept, compute))) return s;
      const tq_status t = tq_check(base + p.table, compute);
      if (t == TQ_EFULL) return t;  // nothing was inserted; the probe matched nothing
      if (t) return t;
    }
    if ((s = tq_check(state, compute))) return s;
    int64_t g = 0;
    TQ_HIP(hipMemcpyAsync(&g, ng, 8, hipMemcpyDeviceToHost, compute));
    TQ_HIP(hipStreamSynchronize(compute));
    g = std::min(g, max_groups);
    res[idx].ngroups = g;
    if (g > 0) {
      std::vector<int64_t> dense((size_t)g * p.nsum);
      std::vector<double> dense_avg((size_t)g * p.nsum);
      TQ_HIP(hipMemcpyAsync(h_keys + idx * max_groups, keys, (size_t)g * 8, hipMemcpyDeviceToHost, compute));
      TQ_HIP(hipMemcpyAsync(h_count + idx * max_groups, count, (size_t)g * 8, hipMemcpyDeviceToHost, compute));
      if (p.nsum) {
        TQ_HIP(hipMemcpyAsync(dense.data(), sums, dense.size() * 8, hipMemcpyDeviceToHost, compute));
        TQ_HIP(hipMemcpyAsync(dense_avg.data(), avg, dense_avg.size() * 8, hipMemcpyDeviceToHost, compute));
      }
      TQ_HIP(hipStreamSynchronize(compute));
      // the caller's layout: [max_groups][TQ_MAX_SUMS] per request
      int64_t* out = h_sums + idx * max_groups * TQ_MAX_SUMS;
      double* out_avg = h_avg + idx * max_groups * TQ_MAX_SUMS;
      for (int64_t k = 0; k < g; k++)
        for (int j = 0; j < p.nsum; j++) {
          out[k * TQ_MAX_SUMS + j] = dense[(size_t)k * p.nsum + j];
          out_avg[k * TQ_MAX_SUMS + j] = dense_avg[(size_t)k * p.nsum + j];
        }
    }
    return TQ_OK;
  }

  void worker(int w) {
    hipStream_t compute = nullptr, copy = nullptr;
    bool ok = hipStreamCreateWithFlags(&compute, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&copy, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      int64_t job, rows;
      size_t off, bytes;
      int split;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return shutdown || slots[w].job >= 0; });
        if (slots[w].job < 0) break;
        job = slots[w].job;
        off = slots[w].off;
        bytes = slots[w].bytes;
        rows = slots[w].rows;
        split = slots[w].split;
      }
      const double start = now_s();
      int64_t kept = -1;
      tq_status s = ok ? execute(reqs[job], arena_base + off, rows, split, compute, copy, job, &kept) : TQ_EHIP;
      if (s) {
        (void)hipStreamSynchronize(compute);
        (void)hipStreamSynchronize(copy);
      }
      // a table too small for the kept rows, sized from the history: run again for the exact
      // count; a partition of a split too large for its table: again with one more split bit
      const bool refit = s == TQ_EFULL && !split && kept > rows && exact[(size_t)job] < 0;
      const bool resplit = s == TQ_EFULL && split && split < kMaxSplitBits;
      {
        std::lock_guard<std::mutex> lk(mu);
        arena.release(off, bytes);
        tq_budget_release(budget, bytes);
        slots[w].job = -1;
        slots[w].busy = false;
        if (first_start[(size_t)job] < 0) first_start[(size_t)job] = start;
        if (refit || resplit) {
          if (refit) exact[(size_t)job] = kept;
          else split_min[(size_t)job] = split + 1;
          retries[(size_t)job]++;
          again.push_back(job);
        } else {
          const tq_request& q = reqs[job];
          if (s == TQ_OK && q.shape != 0 && q.n_dim > 0 && kept >= 0) hist[q.shape].add((double)kept / (double)q.n_dim);
          res[job].start_s = first_start[(size_t)job];
          res[job].worker = w;
          res[job].status = s;
          res[job].reserved_bytes = (int64_t)bytes;
          res[job].retries = retries[(size_t)job];
          res[job].splits = 1 << split;
          res[job].end_s = now_s();
          completed++;
        }
      }
      cv.notify_all();
    }
    if (compute) (void)hipStreamDestroy(compute);
    if (copy) (void)hipStreamDestroy(copy);
  }

  tq_status run(int workers) {
    slots.assign(workers, Slot());
    exact.assign((size_t)n, -1);
    split_min.assign((size_t)n, 0);
    retries.assign((size_t)n, 0);
    first_start.assign((size_t)n, -1.0);
    for (int64_t i = 0; i < n; i++) {
      res[i] = tq_request_result{};
      res[i].status = TQ_OK;
    }
    t0 = Clock::now();
    std::vector<std::thread> th;
    for (int w = 0; w < workers; w++) th.emplace_back([this, w] { worker(w); });
    int64_t next = 0;
    std::unique_lock<std::mutex> lk(mu);
    while (completed < n) {
      // requests to run again come first, then arrivals in order
      const bool rerun = !again.empty();
      if (rerun || next < n) {
        const int64_t job = rerun ? again.front() : next;
        double wait = rerun ? 0.0 : reqs[job].arrival_s - now_s();
        if (wait > 0) {
          cv.wait_for(lk, std::chrono::duration<double>(wait));
          continue;
        }
        int idle = -1;
        for (int w = 0; w < workers && idle < 0; w++)
          if (!slots[w].busy) idle = w;
        if (idle >= 0) {
          int64_t rows = table_rows(job);
          Plan p = plan_of(reqs[job], rows);
          // a join over the capacity (or one whose partition proved too large) runs split:
          // the fewest hash partitions whose table fits
          int split = 0;
          if (reqs[job].shape != 0 && (p.total > tq_budget_cap(budget) || split_min[(size_t)job] > 0)) {
            for (int b = std::max(1, (int)split_min[(size_t)job]); b <= kMaxSplitBits; b++) {
              const Plan pb = plan_of(reqs[job], part_rows(rows, b));
              if (pb.total <= tq_budget_cap(budget)) {
                split = b;
                rows = part_rows(rows, b);
                p = pb;
                break;
              }
            }
          }
          size_t off;
          auto taken = [&] {
            if (rerun) again.pop_front();
            else next++;
          };
          if (p.total > tq_budget_cap(budget)) {  // can never fit: fail it rather than block the queue
            res[job].status = TQ_ENOMEM;
            res[job].retries = retries[(size_t)job];
            res[job].splits = 0;
            res[job].start_s = first_start[(size_t)job] >= 0 ? first_start[(size_t)job] : now_s();
            res[job].end_s = now_s();
            taken();
            completed++;
            continue;
          }
          if (tq_budget_reserve(budget, p.total) == TQ_OK) {
            if (arena.alloc(p.total, &off)) {
              slots[idle] = Slot{job, rows, off, p.total, split, true};
              taken();
              cv.notify_all();
              continue;
            }
            tq_budget_release(budget, p.total);
          }
        }
      }
      cv.wait_for(lk, std::chrono::milliseconds(1));  // a completion frees a worker or memory
    }
    shutdown = true;
    lk.unlock();
    cv.notify_all();
    for (auto& t : th) t.join();
    return TQ_OK;
  }
};

}  // namespace
}  // namespace tq

extern "C" tq_status tq_serve_run(const tq_serve_tables* t, const tq_request* reqs, int64_t n, int32_t workers,
                                  tq_budget* budget, void* d_arena, size_t arena_bytes, int64_t max_groups,
                                  int64_t* h_keys, int64_t* h_count, int64_t* h_sums, double* h_avg,
                                  tq_request_result* res) {
  using tq::fail;
  if (!t || (n > 0 && (!reqs || !res || !h_keys || !h_count || !h_sums || !h_avg)) || !budget || !d_arena)
    return fail(TQ_EINVAL, "NULL argument");
  if (t->fg_rows < 0 || t->dim_rows < 0 || t->fact_rows < 0) return fail(TQ_EINVAL, "negative base table row count");
  if (workers < 1 || workers > 64) return fail(TQ_EINVAL, "workers outside [1, 64]");
  if (max_groups < 1) return fail(TQ_EINVAL, "max_groups");
  for (int64_t i = 0; i < n; i++) {
    const tq_request& q = reqs[i];
    if (i > 0 && q.arrival_s < reqs[i - 1].arrival_s) return fail(TQ_EINVAL, "requests must be in arrival order");
    if (q.shape < 0 || q.shape > 2 || q.n_fact < 0 || q.fact_first < 0) return fail(TQ_EINVAL, "request %lld", (long long)i);
    if (q.shape != 2 && q.fact_first % 16) return fail(TQ_EINVAL, "request %lld: window start not a multiple of 16", (long long)i);
    if (q.shape != 0 && (q.dim_first % 16 || q.n_dim < 0)) return fail(TQ_EINVAL, "request %lld: dimension window", (long long)i);
    if (q.shape == 2 && (!t->pool || q.fact_first + q.n_fact > t->n_fact_batches))
      return fail(TQ_EINVAL, "request %lld: batch window", (long long)i);
    // every window lies inside its base table (a window past the end would make the kernels read past the columns)
    if (q.shape == 0 && q.fact_first + q.n_fact > t->fg_rows)
      return fail(TQ_EINVAL, "request %lld: rows [%lld, %lld) outside the %lld-row filter table", (long long)i,
                  (long long)q.fact_first, (long long)(q.fact_first + q.n_fact), (long long)t->fg_rows);
    if (q.shape == 1 && q.fact_first + q.n_fact > t->fact_rows)
      return fail(TQ_EINVAL, "request %lld: rows [%lld, %lld) outside the %lld-row fact table", (long long)i,
                  (long long)q.fact_first, (long long)(q.fact_first + q.n_fact), (long long)t->fact_rows);
    if (q.shape != 0 && (q.dim_first < 0 || q.dim_first + q.n_dim > t->dim_rows))
      return fail(TQ_EINVAL, "request %lld: rows [%lld, %lld) outside the %lld-row dimension table", (long long)i,
                  (long long)q.dim_first, (long long)(q.dim_first + q.n_dim), (long long)t->dim_rows);
  }
  tq::Server s(*t, reqs, n, budget, d_arena, arena_bytes, max_groups, h_keys, h_count, h_sums, h_avg, res);
  return s.run(workers);
}
