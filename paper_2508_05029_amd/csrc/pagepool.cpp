// Fixed-size page-locked host page pool, batch layout over page chains, the
// host -> device streaming pipeline, and device-memory budget accounting.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"

struct tq_pagepool {
  size_t page_bytes = 0;
  int64_t n_pages = 0;
  char* base = nullptr;
  bool pinned = false;
  std::mutex mu;
  std::vector<int32_t> free_ids;  // a stack of free page ids
};

struct tq_budget {
  size_t cap = 0, used = 0, peak = 0;
  mutable std::mutex mu;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int width_of(int32_t t) { return (t == TQ_U8 || t == TQ_I32 || t == TQ_I64) ? t : 0; }

}  // namespace

extern "C" {

tq_status tq_pagepool_create(size_t page_bytes, int64_t n_pages, uint32_t flags, tq_pagepool** out) {
  using tq::fail;
  if (!out) return fail(TQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (page_bytes == 0 || page_bytes % kAlign) return fail(TQ_EINVAL, "page size %zu is not a multiple of 256", page_bytes);
  if (n_pages <= 0 || n_pages > INT32_MAX) return fail(TQ_EINVAL, "page count %lld", (long long)n_pages);
  if ((size_t)n_pages > SIZE_MAX / page_bytes) return fail(TQ_EINVAL, "pool size overflows");
  size_t total = page_bytes * (size_t)n_pages;
  auto* p = new tq_pagepool();
  p->page_bytes = page_bytes;
  p->n_pages = n_pages;
  p->pinned = !(flags & TQ_POOL_PAGEABLE);
  if (p->pinned) {
    void* mem = nullptr;
    hipError_t e = hipHostMalloc(&mem, total, hipHostMallocDefault);
    if (e != hipSuccess) {
      delete p;
      return fail(TQ_ENOMEM, "pinning %zu bytes failed: %s", total, hipGetErrorString(e));
    }
    p->base = static_cast<char*>(mem);
  } else {
    void* mem = nullptr;
    if (posix_memalign(&mem, 4096, total) != 0) {
      delete p;
      return fail(TQ_ENOMEM, "allocating %zu bytes failed", total);
    }
    p->base = static_cast<char*>(mem);
  }
  p->free_ids.reserve((size_t)n_pages);
  for (int64_t i = n_pages - 1; i >= 0; i--) p->free_ids.push_back((int32_t)i);
  *out = p;
  return TQ_OK;
}

void tq_pagepool_destroy(tq_pagepool* p) {
  if (!p) return;
  if (p->pinned) (void)hipHostFree(p->base);
  else free(p->base);
  delete p;
}

tq_status tq_pagepool_alloc(tq_pagepool* p, int64_t n, int32_t* ids) {
  if (!p || n < 0 || (n > 0 && !ids)) return tq::fail(TQ_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(p->mu);
  if ((int64_t)p->free_ids.size() < n)
    return tq::fail(TQ_ENOMEM, "%lld pages requested, %zu free", (long long)n, p->free_ids.size());
  for (int64_t i = 0; i < n; i++) {
    ids[i] = p->free_ids.back();
    p->free_ids.pop_back();
  }
  return TQ_OK;
}

void tq_pagepool_free(tq_pagepool* p, const int32_t* ids, int64_t n) {
  if (!p || !ids) return;
  std::lock_guard<std::mutex> g(p->mu);
  for (int64_t i = 0; i < n; i++)
    if (ids[i] >= 0 && ids[i] < p->n_pages) p->free_ids.push_back(ids[i]);
}

void* tq_pagepool_page(tq_pagepool* p, int32_t id) {
  if (!p || id < 0 || id >= p->n_pages) return nullptr;
  return p->base + (size_t)id * p->page_bytes;
}

int64_t tq_pagepool_free_pages(tq_pagepool* p) {
  if (!p) return 0;
  std::lock_guard<std::mutex> g(p->mu);
  return (int64_t)p->free_ids.size();
}

size_t tq_pagepool_page_bytes(tq_pagepool* p) { return p ? p->page_bytes : 0; }

}  // extern "C"

namespace tq {

tq_status pool_take_run(tq_pagepool* p, int64_t npages, int32_t* first) {
  if (!p || npages <= 0 || !first) return fail(TQ_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(p->mu);
  // rare (once per out-of-core call): a scan over a map of the free ids
  std::vector<char> is_free((size_t)p->n_pages, 0);
  for (int32_t id : p->free_ids) is_free[(size_t)id] = 1;
  int64_t run = 0, at = -1;
  for (int64_t i = 0; i < p->n_pages; i++) {
    run = is_free[(size_t)i] ? run + 1 : 0;
    if (run == npages) {
      at = i - npages + 1;
      break;
    }
  }
  if (at < 0) return fail(TQ_ENOMEM, "no run of %lld free consecutive pages", (long long)npages);
  p->free_ids.erase(std::remove_if(p->free_ids.begin(), p->free_ids.end(),
                                   [&](int32_t id) { return id >= at && id < at + npages; }),
                    p->free_ids.end());
  *first = (int32_t)at;
  return TQ_OK;
}

void pool_give_run(tq_pagepool* p, int32_t first, int64_t npages) {
  if (!p || first < 0) return;
  std::lock_guard<std::mutex> g(p->mu);
  for (int64_t i = 0; i < npages; i++)
    if (first + i < p->n_pages) p->free_ids.push_back((int32_t)(first + i));
}

}  // namespace tq

extern "C" {

tq_status tq_batch_layout(int64_t nrows, int32_t ncol, const int32_t* types, size_t page_bytes, int64_t* col_offset,
                          size_t* bytes, int64_t* npages) {
  if (nrows < 0 || ncol < 0 || ncol > 64 || (ncol > 0 && (!types || !col_offset)) || page_bytes == 0)
    return tq::fail(TQ_EINVAL, "bad arguments");
  size_t off = 0;
  for (int c = 0; c < ncol; c++) {
    int w = width_of(types[c]);
    if (!w) return tq::fail(TQ_EINVAL, "column %d: bad type", c);
    off = align_up(off, kAlign);
    col_offset[c] = (int64_t)off;
    off += (size_t)nrows * w;
  }
  if (bytes) *bytes = off;
  if (npages) *npages = (int64_t)((off + page_bytes - 1) / page_bytes);
  return TQ_OK;
}

tq_status tq_pagepool_stream(tq_pagepool* pool, const tq_batch* batches, int64_t nb, void* d_staging,
                             size_t staging_bytes, int32_t nslots, tq_batch_fn fn, void* user, hipStream_t copy,
                             hipStream_t compute) {
  using tq::fail;
  if (!pool || (nb > 0 && (!batches || !d_staging || !fn))) return fail(TQ_EINVAL, "bad arguments");
  if (nslots < 1 || nslots > 64) return fail(TQ_EINVAL, "nslots %d outside [1, 64]", nslots);
  const size_t slot_bytes = staging_bytes / nslots / kAlign * kAlign;
  const size_t pb = pool->page_bytes;
  // validate every batch before enqueueing anything
  std::vector<size_t> batch_bytes((size_t)nb);
  for (int64_t i = 0; i < nb; i++) {
    const tq_batch& b = batches[i];
    if (b.ncol < 0 || b.ncol > TQ_MAX_COLS || b.nrows < 0 || b.npages < 0 || (b.npages > 0 && !b.page_ids) ||
        (b.ncol > 0 && (!b.col_offset || !b.col_type)))
      return fail(TQ_EINVAL, "batch %lld: bad descriptor", (long long)i);
    size_t end = 0;
    for (int c = 0; c < b.ncol; c++) {
      int w = width_of(b.col_type[c]);
      if (!w || b.col_offset[c] < 0 || b.col_offset[c] % 16) return fail(TQ_EINVAL, "batch %lld column %d", (long long)i, c);
      end = std::max(end, (size_t)b.col_offset[c] + (size_t)b.nrows * w);
    }
    if (end > (size_t)b.npages * pb) return fail(TQ_EINVAL, "batch %lld: columns exceed its pages", (long long)i);
    if ((size_t)b.npages * pb > slot_bytes)
      return fail(TQ_EINVAL, "batch %lld: %d pages do not fit a %zu-byte staging slot", (long long)i, b.npages, slot_bytes);
    for (int j = 0; j < b.npages; j++)
      if (b.page_ids[j] < 0 || b.page_ids[j] >= pool->n_pages) return fail(TQ_EINVAL, "batch %lld: page id", (long long)i);
    batch_bytes[(size_t)i] = end;
  }
  if (nb == 0) return TQ_OK;
  std::vector<hipEvent_t> copied((size_t)nslots), done((size_t)nslots);
  for (int s = 0; s < nslots; s++) {
    TQ_HIP(hipEventCreateWithFlags(&copied[s], hipEventDisableTiming));
    TQ_HIP(hipEventCreateWithFlags(&done[s], hipEventDisableTiming));
  }
  char* staging = static_cast<char*>(d_staging);
  tq_status st = TQ_OK;
  int64_t issued = 0;
  auto issue_copy = [&](int64_t i) -> tq_status {
    const tq_batch& b = batches[i];
    const int s = (int)(i % nslots);
    char* slot = staging + (size_t)s * slot_bytes;
    if (i >= nslots) TQ_HIP(hipStreamWaitEvent(copy, done[s], 0));  // the slot's previous batch is computed
    size_t left = batch_bytes[(size_t)i];
    for (int j = 0; j < b.npages && left > 0; j++) {
      size_t sz = std::min(left, pb);
      TQ_HIP(hipMemcpyAsync(slot + (size_t)j * pb, pool->base + (size_t)b.page_ids[j] * pb, sz, hipMemcpyHostToDevice, copy));
      left -= sz;
    }
    TQ_HIP(hipEventRecord(copied[s], copy));
    return TQ_OK;
  };
  for (int64_t i = 0; i < nb && st == TQ_OK; i++) {
    // keep up to nslots batches of copies enqueued ahead of the compute side
    while (issued < nb && issued < i + nslots && st == TQ_OK) st = issue_copy(issued++);
    if (st) break;
    const tq_batch& b = batches[i];
    const int s = (int)(i % nslots);
    char* slot = staging + (size_t)s * slot_bytes;
    TQ_HIP(hipStreamWaitEvent(compute, copied[s], 0));
    tq_col cols[TQ_MAX_COLS] = {};
    for (int c = 0; c < b.ncol; c++) {
      cols[c].data = slot + b.col_offset[c];
      cols[c].type = b.col_type[c];
    }
    st = fn(user, i, cols, b.ncol, b.nrows, compute);
    if (st) break;
    TQ_HIP(hipEventRecord(done[s], compute));
  }
  hipError_t e1 = hipStreamSynchronize(copy), e2 = hipStreamSynchronize(compute);
  for (int s = 0; s < nslots; s++) {
    (void)hipEventDestroy(copied[s]);
    (void)hipEventDestroy(done[s]);
  }
  if (st) return st;
  if (e1 != hipSuccess) return tq::hip_fail(e1, "copy stream");
  if (e2 != hipSuccess) return tq::hip_fail(e2, "compute stream");
  return TQ_OK;
}

tq_status tq_budget_create(size_t cap, tq_budget** out) {
  if (!out) return tq::fail(TQ_EINVAL, "out is NULL");
  auto* b = new tq_budget();
  b->cap = cap;
  *out = b;
  return TQ_OK;
}

void tq_budget_destroy(tq_budget* b) { delete b; }

tq_status tq_budget_reserve(tq_budget* b, size_t bytes) {
  if (!b) return tq::fail(TQ_EINVAL, "budget is NULL");
  std::lock_guard<std::mutex> g(b->mu);
  if (bytes > b->cap - b->used)
    return tq::fail(TQ_ENOMEM, "reserving %zu bytes: %zu of %zu in use", bytes, b->used, b->cap);
  b->used += bytes;
  b->peak = std::max(b->peak, b->used);
  return TQ_OK;
}

void tq_budget_release(tq_budget* b, size_t bytes) {
  if (!b) return;
  std::lock_guard<std::mutex> g(b->mu);
  b->used -= std::min(bytes, b->used);
}

size_t tq_budget_used(const tq_budget* b) {
  if (!b) return 0;
  std::lock_guard<std::mutex> g(b->mu);
  return b->used;
}

size_t tq_budget_peak(const tq_budget* b) {
  if (!b) return 0;
  std::lock_guard<std::mutex> g(b->mu);
  return b->peak;
}

size_t tq_budget_cap(const tq_budget* b) { return b ? b->cap : 0; }

}  // extern "C"
