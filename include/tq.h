/*
 * tq — a columnar query hot path for AMD MI355X (gfx950).
 *
 * C ABI of libtq.so. Plain pointers and sizes only.
 *
 * Conventions
 *   d_*      device pointer (HIP global memory) owned by the CALLER
 *   h_*      host pointer owned by the caller
 *   stream   a hipStream_t; work is enqueued on it and every call returns
 *            without synchronising unless its comment says otherwise
 *   columns  Arrow-style fixed-width value buffers (the paper keeps device
 *            batches in Arrow's columnar layout, Section 3.4); a batch is a
 *            set of columns with the same row count (Section 3.1). Device
 *            column pointers must be 16-byte aligned.
 *   errors   argument errors are detected before anything is enqueued and
 *            returned synchronously; errors found by a kernel (a full table,
 *            a group key outside its domain) are latched in the header of the
 *            table or group-by state and returned by tq_check().
 *            tq_last_error() gives the text of the last failure on the
 *            calling thread.
 *   integers all sums and products are int64 with two's-complement wrap
 *            (mod 2^64), so results are independent of the order in which
 *            threads and atomics combine them.
 */
#ifndef TQ_H
#define TQ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */

typedef int32_t tq_status;
#define TQ_OK 0
#define TQ_EINVAL (-1)   /* bad argument, detected before enqueueing */
#define TQ_ENOMEM (-2)   /* page pool or device budget exhausted */
#define TQ_EFULL (-3)    /* hash table or output capacity too small */
#define TQ_EDOMAIN (-4)  /* a group key fell outside [0, domain) */
#define TQ_EHIP (-5)     /* a HIP runtime call failed */

const char* tq_strerror(tq_status s);
const char* tq_last_error(void); /* thread-local; "" when none */
int32_t tq_version(void);

/* --------------------------------------------------------- row descriptors */

typedef enum { TQ_U8 = 1, TQ_I32 = 4, TQ_I64 = 8 } tq_type; /* values widen to int64 */

typedef struct {
  const void* data;     /* d_ column values */
  int32_t type;         /* tq_type */
  const uint8_t* valid; /* d_ validity bitmap or NULL (no NULLs): bit r of byte r / 8, least significant
                           bit first, 1 = value present (the Arrow layout, Section 3.4). Only the *_nullable
                           entry points accept columns that carry one (the others return TQ_EINVAL). */
} tq_col;

/* lo <= col <= hi on the widened value; a list of predicates is a conjunction. */
typedef struct {
  int32_t col;
  int64_t lo, hi;
} tq_pred;

/* sign * col + add; col = -1 means the constant `add`. */
typedef struct {
  int32_t col;
  int32_t sign;
  int64_t add;
} tq_factor;

/* Product of nf (1..3) factors, evaluated left to right in int64 mod 2^64. */
typedef struct {
  int32_t nf;
  tq_factor f[3];
} tq_expr;

/* Group key: col[0] * mult + col[1] (ncol = 2) or col[0] (ncol = 1). */
typedef struct {
  int32_t ncol;
  int32_t col[2];
  int64_t mult;
} tq_gkey;

#define TQ_MAX_COLS 8
#define TQ_MAX_PREDS 4
#define TQ_MAX_SUMS 6

/* ---------------------------------------------------- filter and project */

/* Selection and projection (the Filter operator of Section 3.1 and the
 * per-task computation of Section 3.3.1). For every row of `in` that
 * satisfies all `np` predicates, writes the `ne` expression values to
 * d_out[e][i] and, if d_sel is not NULL, the source row index to d_sel[i],
 * for i < *d_out_rows, in ascending row order (a stable compaction). Each
 * output must hold nrows values. *d_out_rows (device) is set by the call.
 * d_scratch (device) must hold tq_filter_project_scratch_bytes(nrows) bytes
 * and must not be shared by calls that overlap. */
size_t tq_filter_project_scratch_bytes(int64_t nrows);
tq_status tq_filter_project(const tq_col* in, int32_t ncol, int64_t nrows, const tq_pred* p, int32_t np,
                            const tq_expr* e, int32_t ne, int64_t* const* d_out, int64_t* d_sel,
                            int64_t* d_out_rows, void* d_scratch, size_t scratch_bytes, hipStream_t stream);

/* ------------------------------------------------------------ hash partition */

/* Hash partitioning, the exchange in front of a join (Section 3.2): row r goes
 * to partition p(r) = bits [skip, skip + log2_fanout) counted from the most
 * significant end of h = key_r * 0x9E3779B97F4A7C15 (mod 2^64). Writes the
 * keys and every payload column partition by partition (partition p occupies
 * rows d_offsets[p] .. d_offsets[p+1]-1; d_offsets has 2^log2_fanout + 1
 * entries); the order inside a partition is unspecified. Payload columns keep
 * their type. Needs a device scratch buffer of
 * tq_hash_partition_scratch_bytes(n, log2_fanout) bytes. log2_fanout <= 10,
 * skip + log2_fanout <= 64. */
size_t tq_hash_partition_scratch_bytes(int64_t n, int32_t log2_fanout);
tq_status tq_hash_partition(const int64_t* d_keys, const tq_col* payload, int32_t npay, int64_t n,
                            int32_t log2_fanout, int32_t skip, int64_t* d_out_keys, void* const* d_out_payload,
                            int64_t* d_offsets, void* d_scratch, size_t scratch_bytes, hipStream_t stream);

/* tq_hash_partition for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc): the
 * same partitioning and outputs, with the scratch taken from a fixed array in
 * the library's device image (TQ_PARTITION_STATIC_SCRATCH_BYTES per GPU, held
 * until the process ends) instead of a caller buffer. The call allocates
 * nothing; it looks the array's address up on its first call on each device
 * (the calling thread's current device must be the one `stream` belongs to).
 * A size whose scratch (tq_hash_partition_scratch_bytes(n, log2_fanout))
 * exceeds the array returns TQ_EINVAL before anything is enqueued. Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be serialised by
 * the caller. */
#define TQ_PARTITION_STATIC_SCRATCH_BYTES (8u << 20)
tq_status tq_hash_partition_noalloc(const int64_t* d_keys, const tq_col* payload, int32_t npay, int64_t n,
                                    int32_t log2_fanout, int32_t skip, int64_t* d_out_keys,
                                    void* const* d_out_payload, int64_t* d_offsets, hipStream_t stream);

/* ------------------------------------------------------------- hash join */

/* An open-addressing hash table (linear probing over buckets of 8 slots) for
 * the build side of an equi-join (the Adaptive Join of Section 3.2). Layout: a
 * 256-byte header, a 16 KiB area of per-workgroup partial counts, a 16-bit tag
 * per slot (0 = empty), a 16-byte {key, payload} slot array, and a build
 * scratch area of about the slot array's size (the rows grouped by table
 * region, alternate tags for a fallback build, and a Bloom filter of the keys
 * that probes use to skip rows with no partner, two bits per slot for tables
 * built region by region). A build fills the table region by region in LDS
 * (256 regions; past 2^19 slots each region as domains of 2048 slots, one
 * after the other), or,
 * past 2^23 slots or when some region or domain gets more rows than it holds
 * with an eighth free, inserts with global atomics.
 * Any int64 key is allowed; duplicate build keys are kept (many-to-many).
 * tq_join_table_bytes gives the size for at most n_build_max rows at the given
 * load factor (0 < load_factor <= 0.9). The capacity actually used by a build
 * is the smallest power of two >= rows / load_factor, computed on the device
 * from the number of rows that pass the build filter. */
size_t tq_join_table_bytes(int64_t n_build_max, double load_factor);

/* Prepare a table buffer once after allocation (zeroes its header). */
tq_status tq_join_table_init(void* d_table, size_t bytes, hipStream_t stream);

#define TQ_UNIQUE_KEYS 1u /* build keys are unique: a probe stops at its first match */
/* One hash partition of a join (the split of a task that does not fit its
 * memory, Section 3.3.2): with TQ_SELECT_PARTITION | TQ_PARTITION(id) in the
 * build's flags and 1 <= skip <= 16, the build keeps only the rows whose key
 * hash (key * 0x9E3779B97F4A7C15 mod 2^64) has `id` in its top `skip` bits,
 * and every probe of the table then takes only the probe rows of that
 * partition (the others match nothing). Running the 2^skip partitions one after
 * another into one group-by state gives the whole join's result, each with a
 * table sized for its share of the rows. */
#define TQ_SELECT_PARTITION 2u
#define TQ_PARTITION(id) ((uint32_t)(id) << 16)

/* Build: insert (keys[r], payload[r]) for every row r < n that satisfies the
 * optional predicates over `filt` (the dimension filter fused into the build).
 * `skip` high hash bits are ignored by the slot index (set it to the partition
 * bits when the input is one hash partition). Latches TQ_EFULL if the rows do
 * not fit in the buffer; the header still records how many rows passed the
 * filter (tq_join_table_rows), and nothing is inserted. Every build replaces
 * the previous one, an error it latched included. Three or four kernel
 * launches on `stream`, none of which allocates; builds into one buffer must
 * not overlap. */
tq_status tq_join_build(void* d_table, size_t bytes, const int64_t* d_keys, tq_col payload, int64_t n,
                        const tq_col* filt, int32_t nfilt, const tq_pred* p, int32_t np, double load_factor,
                        int32_t skip, uint32_t flags, hipStream_t stream);

/* Rows that passed the last build's filter, read from a table's header after
 * the build has completed (synchronises `stream`); set even when the build
 * latched TQ_EFULL. */
tq_status tq_join_table_rows(const void* d_table, int64_t* rows, hipStream_t stream);

/* Fused group-by applied to probe matches: group key = the matched build
 * payload, sums = expressions over the probe-side columns passed to
 * tq_join_probe. d_state comes from tq_groupby_init. */
typedef struct {
  void* d_state;
  int64_t domain; /* as passed to tq_groupby_init (or tq_groupby_init_nullable) */
  const tq_expr* sums;
  int32_t nsum;   /* as passed to tq_groupby_init (or tq_groupby_init_nullable) */
  int32_t nullable; /* 1: d_state comes from tq_groupby_init_nullable (tq_join_probe_nullable only) */
} tq_agg;

/* Probe: for every probe row r < n that satisfies the optional predicates over
 * `cols`, find every build slot with key == d_probe_keys[r].
 *   agg == NULL  write pairs (r, payload) to d_out_probe_row / d_out_payload
 *                in ascending probe-row order (the matches of one row in
 *                slot order), at most `capacity` of them; *d_out_count gets
 *                the total match count, which may exceed capacity (then the
 *                pairs past `capacity` are dropped; the caller compares).
 *                Uses the table's partial-count area: materialising probes
 *                of one table must not overlap.
 *   agg != NULL  aggregate the matches into agg->d_state instead (the
 *                state's COUNT column counts them); the pair outputs and
 *                d_out_count must be NULL.
 * A table whose build latched an error matches nothing. */
tq_status tq_join_probe(const void* d_table, const int64_t* d_probe_keys, int64_t n, const tq_col* cols,
                        int32_t ncol, const tq_pred* p, int32_t np, int64_t* d_out_probe_row,
                        int64_t* d_out_payload, int64_t capacity, int64_t* d_out_count, const tq_agg* agg,
                        hipStream_t stream);

/* The join under NULLs: a NULL key (d_key_valid, a bitmap or NULL; build or
 * probe side) equals nothing; the build's filter columns and payload may carry
 * bitmaps, and a NULL payload is stored as INT64_MIN (a payload column with
 * NULLs must not hold INT64_MIN itself). The probe aggregates into a nullable
 * group-by state (agg->nullable = 1, from tq_groupby_init_nullable): a match
 * whose payload is NULL goes to the NULL group, and a probe value that is NULL
 * makes the sums reading it skip the row. Arguments as tq_join_build and the
 * fused tq_join_probe otherwise. */
tq_status tq_join_build_nullable(void* d_table, size_t bytes, const int64_t* d_keys, const uint8_t* d_key_valid,
                                 tq_col payload, int64_t n, const tq_col* filt, int32_t nfilt, const tq_pred* p,
                                 int32_t np, double load_factor, int32_t skip, uint32_t flags, hipStream_t stream);
tq_status tq_join_probe_nullable(const void* d_table, const int64_t* d_probe_keys, const uint8_t* d_key_valid,
                                 int64_t n, const tq_col* cols, int32_t ncol, const tq_pred* p, int32_t np,
                                 const tq_agg* agg, hipStream_t stream);

/* --------------------------------------------- string keys (dictionaries) */

/* A column of strings in Arrow's layout: string i is the bytes
 * data[offsets[i] .. offsets[i + 1]) (offsets: n + 1 int32 entries). */
typedef struct {
  const int32_t* offsets; /* d_ */
  const uint8_t* data;    /* d_ */
  int64_t n;
} tq_strings;

/* String join and group keys are dictionary-encoded (the Arrow dictionary
 * arrays of the columnar layout, Section 3.4): int32 codes into a dictionary of
 * distinct strings. Grouping by a string column groups by its codes (domain =
 * the dictionary size; the caller decodes the output keys). Joining two string
 * columns encoded against different dictionaries maps the probe side's
 * dictionary onto the build side's: tq_dict_unify sets d_remap[i] = the index
 * j of the build dictionary entry equal byte for byte to probe dictionary
 * entry i, or -1 if there is none. The build dictionary's entries must be
 * distinct. d_table is a join table buffer for build.n rows
 * (tq_join_table_bytes(build.n, 0.5)), d_scratch holds
 * tq_dict_unify_scratch_bytes(build.n) bytes; both are overwritten. */
size_t tq_dict_unify_scratch_bytes(int64_t n_build);
tq_status tq_dict_unify(void* d_table, size_t table_bytes, tq_strings build, tq_strings probe, void* d_scratch,
                        size_t scratch_bytes, int32_t* d_remap, hipStream_t stream);

/* Dictionary encoding of a plain string column (its strings need not be
 * distinct): d_codes[i] = the code of string i, equal codes exactly for equal
 * strings; codes are 0 .. *d_ndict - 1 (numbered in the order of a 64-bit
 * hash of the bytes, FNV-1a), and d_first_rows[c] = the smallest row holding
 * code c, from which the dictionary's strings are read. A group-by or a join
 * on strings then runs on the codes (both sides of a join encoded as one
 * column). d_codes and d_first_rows hold n entries; d_scratch
 * tq_dict_encode_scratch_bytes(n) bytes (temporary storage of a radix sort by
 * hash, and run tables). *d_ndict is written on the device, -1 if more than 16
 * distinct strings shared one hash. n < 2^31 - 1. */
size_t tq_dict_encode_scratch_bytes(int64_t n);
tq_status tq_dict_encode(tq_strings in, void* d_scratch, size_t scratch_bytes, int32_t* d_codes, int32_t* d_first_rows,
                         int64_t* d_ndict, hipStream_t stream);

/* int64 join keys from dictionary codes: d_keys[r] = codes[r] (d_remap NULL)
 * or d_remap[codes[r]], and -1 where the code is NULL (d_valid, a bitmap or
 * NULL), outside [0, n_remap) or maps to no entry. Codes of the build side
 * (>= 0) never equal -1, so a probe key of -1 matches nothing; build rows whose
 * code is NULL are left out by tq_join_build_nullable with the same bitmap. */
tq_status tq_dict_keys(const int32_t* d_codes, const uint8_t* d_valid, int64_t n, const int32_t* d_remap,
                       int64_t n_remap, int64_t* d_keys, hipStream_t stream);

/* ------------------------------------------------------------- group-by */

/* Group-by state for keys in [0, domain) with COUNT and `nsum` int64 SUMs
 * (the aggregations of Section 2). It accumulates across any number of
 * tq_groupby_agg / fused-probe calls (batches, partitions, requests). Calls
 * that update one state must not overlap (issue them on one stream). Small
 * domains (domain * (1 + nsum) <= 1024) keep one private partial row per
 * workgroup, folded by tq_groupby_finalize; larger ones one shared table. */
size_t tq_groupby_state_bytes(int64_t domain, int32_t nsum);
tq_status tq_groupby_init(void* d_state, size_t bytes, int64_t domain, int32_t nsum, hipStream_t stream);

/* Accumulate the rows of `in` that satisfy the predicates: key from `key`
 * (must lie in [0, domain), else TQ_EDOMAIN is latched and the row dropped),
 * COUNT += 1 and SUM_j += sums[j](row). `domain` and `nsum` must be the values
 * the state was initialised with; if they are not, the kernel writes nothing
 * and latches TQ_EINVAL. */
tq_status tq_groupby_agg(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                         const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                         hipStream_t stream);

/* Emit the groups with COUNT > 0 in ascending key order: d_keys[g],
 * d_count[g], d_sums[g * nsum + j] and, if d_avg is not NULL,
 * d_avg[g * nsum + j] = (double)SUM_j / (double)COUNT (IEEE round to nearest
 * even). Outputs must hold `domain` groups; *d_ngroups gets the count. */
tq_status tq_groupby_finalize(const void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums,
                              double* d_avg, int64_t* d_ngroups, hipStream_t stream);

/* tq_groupby_finalize that also leaves the state empty, as tq_groupby_init
 * does (every partial it read is zeroed in the same pass), so that a caller
 * running one query after another on a state skips the separate set-up: the
 * next aggregation starts from zero. A latched error stays latched (it is
 * reported by tq_check and cleared by tq_groupby_init). */
tq_status tq_groupby_finalize_reset(void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums, double* d_avg,
                                    int64_t* d_ngroups, hipStream_t stream);

/* NULLs (SQL's semantics over Arrow validity bitmaps, the columnar layout of
 * Section 3.4): a predicate over a NULL value is not true, so the row is
 * dropped; a sum whose expression reads a NULL value skips the row; COUNT(*)
 * counts every row; rows whose group key is NULL form one group of their own.
 * A nullable state for keys in [0, domain) keeps, per group and per sum j,
 * SUM_j and COUNT_j (the rows where sum j is not NULL), and one more group for
 * the NULL key; at most 3 sums. tq_groupby_agg_nullable takes the arguments of
 * tq_groupby_agg; its group key has one column. tq_groupby_finalize_nullable
 * emits the groups with COUNT(*) > 0 in ascending key order, the NULL group
 * last with d_keys[g] = domain (the key that stands for NULL), d_sums[g * nsum
 * + j] = SUM_j, d_nonnull[g * nsum + j] = COUNT_j (SUM_j and AVG_j are NULL when
 * it is 0, and are then written as 0), d_avg = (double)SUM_j / (double)COUNT_j.
 * Outputs must hold domain + 1 groups. */
size_t tq_groupby_state_bytes_nullable(int64_t domain, int32_t nsum);
tq_status tq_groupby_init_nullable(void* d_state, size_t bytes, int64_t domain, int32_t nsum, hipStream_t stream);
tq_status tq_groupby_agg_nullable(void* d_state, int64_t domain, const tq_col* in, int32_t ncol, int64_t nrows,
                                  const tq_pred* p, int32_t np, const tq_gkey* key, const tq_expr* sums, int32_t nsum,
                                  hipStream_t stream);
tq_status tq_groupby_finalize_nullable(const void* d_state, int64_t* d_keys, int64_t* d_count, int64_t* d_sums,
                                       int64_t* d_nonnull, double* d_avg, int64_t* d_ngroups, hipStream_t stream);

/* Synchronise `stream`, then return the error latched in a join table, a
 * group-by state or a Parquet decode's work buffer (TQ_OK if none). */
tq_status tq_check(const void* d_obj, hipStream_t stream);

/* ------------------------------------------------------------ page pool */

/* A pool of fixed-size page-locked host pages, allocated once when the pool is
 * created (the fixed-size page-locked buffer pool of Section 3.4; the paper
 * found per-request pinned allocation slow and fragmenting). Batches are laid
 * out over chains of pages: the columns of a batch follow each other in the
 * chain's byte stream, each starting 256-byte aligned, and may straddle page
 * boundaries; the tail of the last page is unused. Pages also serve as spill
 * targets and staging buffers. Thread-safe. */
typedef struct tq_pagepool tq_pagepool;

#define TQ_POOL_PAGEABLE 1u /* ordinary host memory instead of pinned (no GPU needed; slower copies) */

tq_status tq_pagepool_create(size_t page_bytes, int64_t n_pages, uint32_t flags, tq_pagepool** out);
void tq_pagepool_destroy(tq_pagepool* pool);
/* Take n pages (all or nothing): page ids to h_page_ids; TQ_ENOMEM if fewer are free. */
tq_status tq_pagepool_alloc(tq_pagepool* pool, int64_t n, int32_t* h_page_ids);
void tq_pagepool_free(tq_pagepool* pool, const int32_t* h_page_ids, int64_t n);
void* tq_pagepool_page(tq_pagepool* pool, int32_t id); /* host address of a page; NULL if id is invalid */
int64_t tq_pagepool_free_pages(tq_pagepool* pool);
size_t tq_pagepool_page_bytes(tq_pagepool* pool);

/* Column offsets of a batch of `nrows` rows with the given column types in a
 * page chain: h_col_offset[c] (bytes from the start of the chain), the bytes
 * the batch occupies (*h_bytes) and the pages it needs (*h_npages). */
tq_status tq_batch_layout(int64_t nrows, int32_t ncol, const int32_t* h_types, size_t page_bytes,
                          int64_t* h_col_offset, size_t* h_bytes, int64_t* h_npages);

typedef struct {
  int32_t npages;
  const int32_t* page_ids; /* the chain */
  int64_t nrows;
  int32_t ncol;
  const int64_t* col_offset; /* from tq_batch_layout */
  const int32_t* col_type;
} tq_batch;

/* Called once per batch, on the calling thread, after the batch's copy has
 * been enqueued: `d_cols` point into the device staging slot that will hold
 * the batch once `compute` reaches the work enqueued next, so the callback
 * enqueues its kernels on `compute` and returns. A non-OK return stops the
 * stream and is returned by tq_pagepool_stream. */
typedef tq_status (*tq_batch_fn)(void* user, int64_t batch_idx, const tq_col* d_cols, int32_t ncol,
                                 int64_t nrows, hipStream_t compute);

/* Stream batches host -> device with the copies overlapped with compute
 * (compute-task pre-loading, Section 3.3.3): batch i is copied page by page
 * into staging slot i mod nslots on `copy` (so straddling columns become
 * contiguous on the device) while earlier batches compute on `compute`; a
 * slot is refilled only after the compute work of the batch it held is done.
 * d_staging holds nslots slots of staging_bytes / nslots bytes each (a slot
 * must hold the largest batch, rounded to whole pages). Blocks until every
 * copy and every callback's compute work has completed (both streams are
 * synchronised before it returns). */
tq_status tq_pagepool_stream(tq_pagepool* pool, const tq_batch* batches, int64_t nb, void* d_staging,
                             size_t staging_bytes, int32_t nslots, tq_batch_fn on_resident, void* user,
                             hipStream_t copy, hipStream_t compute);

/* ------------------------------------------------------------ budget */

/* Device-memory reservations (Section 3.3.2): a task reserves before it
 * allocates; a reservation that does not fit returns TQ_ENOMEM (the caller
 * then spills and retries). Thread-safe, host-only accounting. */
typedef struct tq_budget tq_budget;
tq_status tq_budget_create(size_t cap_bytes, tq_budget** out);
void tq_budget_destroy(tq_budget* b);
tq_status tq_budget_reserve(tq_budget* b, size_t bytes);
void tq_budget_release(tq_budget* b, size_t bytes);
size_t tq_budget_used(const tq_budget* b);
size_t tq_budget_peak(const tq_budget* b);
size_t tq_budget_cap(const tq_budget* b);

/* ------------------------------------------------------------ out-of-core join */

/* The out-of-core join + aggregate (Section 3.2's exchange in front of a
 * join, run on one GPU). Both sides stream from page-pool batches
 * (tq_pagepool_stream); the dimension is filtered first, then the fact side
 * follows.
 *
 * Adaptive Exchange (Section 3.2): the exchange in front of the join does not
 * wait for its whole input before it chooses how to move it. Once the first
 * dimension batches holding at least an eighth of the dimension's rows have
 * been filtered, the kept fraction of those rows estimates the filtered
 * dimension's size, and the exchange chooses one of two modes (plan.exchange
 * may force either):
 *  - single: one join table over every kept dimension row fits the budget, so
 *    the fact side is not exchanged at all. Each staged fact batch probes that
 *    table straight from its staging slot, aggregating as it goes: no fact
 *    partitioning, no holders, no spills, no second pass. (On one GPU this is
 *    what broadcasting the build side amounts to.)
 *  - partitioned: both sides are hash partitioned into 2^log2_fanout
 *    partitions whose rows are appended to per-partition holders of
 *    fixed-size device chunks reserved from `budget`. When a reservation
 *    fails, the resident chunks of the partition scheduled latest are copied
 *    to pool pages (device -> host, on a stream of their own) and released
 *    (Section 3.3.2: spill the data whose compute is furthest away). Pass 2
 *    joins partition by partition in order, reloading spilled chunks one
 *    partition ahead of use, and aggregates into `agg`.
 * Dimension rows filtered before the choice are hash partitioned, so either
 * mode can use them. When the exact kept count at the end of the dimension
 * side shows that an automatic single choice no longer fits, the dimension's
 * holders are released and the dimension side is streamed again,
 * partitioned (stats.dim_restreams counts this). The group key is the
 * dimension payload column. All library device memory counts against the
 * budget. */
#define TQ_EXCHANGE_AUTO 0        /* choose from the estimate */
#define TQ_EXCHANGE_PARTITIONED 1 /* always hash partition both sides */
#define TQ_EXCHANGE_SINGLE 2      /* always one table (TQ_ENOMEM if it does not fit) */
typedef struct {
  int32_t dim_key_col;     /* int64 */
  int32_t dim_payload_col; /* group id */
  const tq_pred* dim_preds;
  int32_t dim_np;
  int32_t fact_key_col;    /* int64 */
  int32_t fact_keep_mask;  /* fact columns carried through the exchange (bit c = column c; must
                              include the key and every column the sums read) */
  const tq_expr* sums;     /* over fact column indices */
  int32_t nsum;
  int64_t domain;
  int32_t log2_fanout;     /* <= 10 */
  double load_factor;
  uint32_t join_flags;     /* TQ_UNIQUE_KEYS when the dimension keys are unique */
  size_t chunk_bytes;      /* device holder chunk size, a divisor of the pool's page size */
  int32_t nslots;          /* staging slots of the streaming passes (>= 2) */
  int32_t exchange;        /* TQ_EXCHANGE_AUTO, _PARTITIONED or _SINGLE */
} tq_ooc_plan;

typedef struct {
  int64_t bytes_h2d, bytes_d2h;      /* bytes copied by the streaming passes, spills and reloads */
  int64_t spilled_chunks, reloaded_chunks;
  int64_t dim_rows_kept, fact_rows;
  int64_t peak_budget_bytes;
  double ms_pass1, ms_pass2, ms_total; /* host wall clock; single mode: pass 1 = dimension side and
                                          table build, pass 2 = fact side */
  int32_t exchange;                    /* the mode used: TQ_EXCHANGE_PARTITIONED or TQ_EXCHANGE_SINGLE */
  int32_t dim_restreams;               /* times the dimension side was streamed again */
  int64_t est_dim_rows;                /* the estimate of kept dimension rows (0 when the mode was forced) */
  int64_t est_from_rows;               /* dimension rows filtered when the estimate was taken */
} tq_ooc_stats;

/* d_work: the device memory the call may use (work_bytes >= the budget's
 * capacity is not required: the call never uses more than the smaller of the
 * two). d_state: a group-by state initialised by the caller for
 * (domain, nsum); the call accumulates into it and leaves finalization to the
 * caller. Spilled chunks use free pool pages. Blocks until the work is done.
 * Returns TQ_ENOMEM if the budget cannot hold the fixed buffers plus one
 * partition's working set, or the pool has no page left to spill to, or a
 * forced single table does not fit. */
tq_status tq_ooc_join_agg(tq_pagepool* pool, const tq_batch* dim, int64_t n_dim_batches, const tq_batch* fact,
                          int64_t n_fact_batches, const tq_ooc_plan* plan, tq_budget* budget, void* d_work,
                          size_t work_bytes, void* d_state, tq_ooc_stats* stats, hipStream_t copy,
                          hipStream_t compute);

/* ------------------------------------------------------------ batched instances */

/* Many independent join + group-by instances of one query shape (the
 * task-on-batch model of Section 3.1 taken to thousands of small, uneven
 * batches). Dimension columns: [0] the int64 key, [1] the group id, the rest
 * filter columns; fact columns: [0] the int64 foreign key, the rest read by
 * the sums. Per instance the caller provides the table, the group-by state and
 * the outputs; tile sizes and the load factor are per instance (autotuned by
 * size bucket). */
typedef struct {
  int32_t dim_types[4];
  int32_t ndim;
  tq_pred preds[2]; /* the build filter, over dimension columns */
  int32_t np;
  int32_t fact_types[4];
  int32_t nfact;
  tq_expr sums[2]; /* over fact columns */
  int32_t nsum;
  uint32_t join_flags; /* TQ_UNIQUE_KEYS */
} tq_batch_query;

typedef struct {
  const void* dim_cols[4];
  int64_t n_dim;
  const void* fact_cols[4];
  int64_t n_fact;
  int64_t domain;     /* group ids lie in [0, domain) */
  void* d_table;      /* tq_join_table_bytes(n_dim, load_factor) bytes */
  size_t table_bytes;
  void* d_state;      /* tq_batched_state_bytes(domain, nsum) bytes */
  size_t state_bytes;
  int64_t* d_keys;    /* outputs: `domain` entries each (sums, avg: domain * nsum) */
  int64_t* d_count;
  int64_t* d_sums;
  double* d_avg;
  int64_t* d_ngroups;
  double load_factor;
  int32_t build_tile; /* rows per build work item */
  int32_t probe_tile; /* rows per probe work item */
} tq_instance;

size_t tq_batched_state_bytes(int64_t domain, int32_t nsum);
/* Device work area for n instances (descriptors, the work-item list, counters,
 * and each instance's Bloom filter of its kept build keys: 2 bits per build
 * row, 256 B to 32 KiB). */
size_t tq_batched_work_bytes(const tq_instance* h_inst, int32_t n);

/* Upload the descriptors and the work-item list for tq_batched_run (copies
 * synchronously; not part of the timed work). */
tq_status tq_batched_prepare(const tq_batch_query* q, const tq_instance* h_inst, int32_t n, void* d_work,
                             size_t work_bytes, hipStream_t stream);

/* One pass over the n prepared instances: a preparation kernel (table headers,
 * tags, states, counters), then one persistent launch per phase (build tiles;
 * probe tiles; single-chunk finalizes and chunk counts; chunk writes) whose
 * workgroups take the phase's work items of all instances from an atomic
 * queue. An item needs only earlier phases, so no workgroup waits for
 * another. Only kernels are enqueued, so the call can be captured in a
 * hipGraph and replayed. tq_batched_check synchronises `stream` and reports an
 * error latched in the work area by the last run. */
tq_status tq_batched_run(const tq_batch_query* q, void* d_work, int32_t n, hipStream_t stream);
tq_status tq_batched_check(const void* d_work, hipStream_t stream);

/* The same work as separate stand-alone calls, one build, probe and finalize
 * launch per instance (the baseline the batched launches are compared with). */
tq_status tq_batched_run_per_instance(const tq_batch_query* q, const tq_instance* h_inst, int32_t n,
                                      hipStream_t stream);

/* ------------------------------------------------------------ serving */

/* A request loop over three query templates (shape 0: filter + group-by over
 * a device table; shape 1: join + group-by over device tables; shape 2: the
 * same join with the fact rows streamed from page-pool batches). A request
 * is a row window of the shape's base tables. Requests are admitted in
 * arrival order when their device memory (table, group-by state, outputs,
 * staging) can be reserved from the budget (Section 3.3.2), then run on one
 * of `workers` worker threads, each with its own HIP streams, so requests
 * that arrive while others run overlap on the device; their tables and
 * partial aggregates stay resident until they complete. workers = 1 is the
 * one-at-a-time FIFO baseline.
 *
 * Reservations (Section 3.3.2): a join request's table is sized for the rows
 * its dimension window keeps after the filter. With estimate = 0 that is the
 * whole window (the worst case). With estimate = 1 each shape keeps a history
 * of the kept fraction of its last 16 completed joins, and a request reserves
 * a table for its window times the largest of those fractions, plus a quarter
 * and 1024 rows (the worst case while the history is empty). A request whose
 * table then proves too small (the build latches TQ_EFULL and has recorded
 * the exact kept count) releases its reservation and is queued again ahead
 * of new arrivals, reserving for that exact count; its result counts the
 * retry. Work is not split into smaller tasks. */
typedef struct {
  int32_t shape;     /* 0, 1 or 2 */
  int64_t fact_first; /* shapes 0, 1: first row (a multiple of 16); shape 2: first batch */
  int64_t n_fact;     /* shapes 0, 1: rows; shape 2: batches */
  int64_t dim_first, n_dim; /* shapes 1, 2: dimension window (first a multiple of 16) */
  double arrival_s;  /* arrival time, seconds after the start of the run */
} tq_request;

typedef struct {
  /* shape 0 */
  tq_col fg_cols[TQ_MAX_COLS];
  int32_t fg_ncol;
  tq_pred fg_preds[TQ_MAX_PREDS];
  int32_t fg_np;
  tq_gkey fg_key;
  tq_expr fg_sums[TQ_MAX_SUMS];
  int32_t fg_nsum;
  int64_t fg_domain;
  /* shapes 1 and 2: dimension (device) = key, payload, filter columns */
  tq_col dim_cols[4];
  int32_t dim_ncol;
  tq_pred dim_preds[2];
  int32_t dim_np;
  /* shape 1: fact (device) = key, then the columns the sums read */
  tq_col fact_cols[4];
  int32_t fact_ncol;
  tq_expr join_sums[2];
  int32_t join_nsum;
  int64_t join_domain;
  double load_factor;
  /* shape 2: fact batches in `pool`; fact_map[j] = batch column of fact column j */
  tq_pagepool* pool;
  const tq_batch* fact_batches;
  int64_t n_fact_batches;
  int32_t fact_map[4];
  int32_t nslots;
  int32_t estimate; /* 1: reserve join tables from the memory-use history; 0: for the whole window */
  /* rows of the base tables: every request window must lie inside them (else TQ_EINVAL) */
  int64_t fg_rows;   /* shape 0 table */
  int64_t dim_rows;  /* dimension (shapes 1, 2) */
  int64_t fact_rows; /* shape 1 fact table */
} tq_serve_tables;

typedef struct {
  double start_s, end_s; /* run on a worker from .. results on the host at */
  int32_t status;        /* TQ_OK or the error of the request */
  int32_t worker;
  int64_t ngroups;
  int64_t reserved_bytes; /* the device memory of the run that completed it */
  int32_t retries;        /* runs that ended with a table too small for the kept rows */
  int32_t splits;         /* hash partitions its join ran as, one after another (1: whole) */
} tq_request_result;

/* Runs all requests and blocks until they are done. d_arena / arena_bytes is
 * the device memory requests are carved from; the budget bounds it. Group
 * results of request i go to h_keys[i][max_groups], h_count[i][max_groups],
 * h_sums[i][max_groups][TQ_MAX_SUMS] (sum j of group g at g * TQ_MAX_SUMS + j)
 * and h_avg (same layout: (double)SUM_j / (double)COUNT, rounded to nearest
 * even), groups in key order, at most max_groups of them; per-request timing
 * to `res`.
 *
 * What a request reserves: the sum, each rounded up to 256 bytes (and at
 * least 8), of tq_groupby_state_bytes(domain, nsum), the join table
 * (tq_join_table_bytes(rows, load_factor), shapes 1 and 2; 0 for shape 0),
 * keys and COUNT (8 * domain each), SUMs and AVGs (8 * domain * nsum each),
 * the group count (8), the staging slots of shape 2 (nslots times the largest
 * batch of its window in whole pages; 0 otherwise) and 64 bytes of scratch.
 * A join request whose reservation exceeds the budget's capacity is split
 * (the third remedy of Section 3.3.2): it runs as 2^b hash partitions one
 * after another (TQ_SELECT_PARTITION builds over its whole windows, each
 * followed by the probe of the whole fact window, all into one group-by
 * state), with the smallest b <= 8 whose table, sized for a 2^-b share of the
 * rows plus a quarter and 1024 rows, fits; a partition that proves larger than
 * its table runs the request again with one more split bit. A request that
 * cannot fit even so (or a filter + group-by request over the capacity)
 * completes at once with status TQ_ENOMEM; the others wait for room.
 * Every window is checked against the base tables' row counts before any
 * request runs (TQ_EINVAL). */
tq_status tq_serve_run(const tq_serve_tables* t, const tq_request* reqs, int64_t n, int32_t workers,
                       tq_budget* budget, void* d_arena, size_t arena_bytes, int64_t max_groups, int64_t* h_keys,
                       int64_t* h_count, int64_t* h_sums, double* h_avg, tq_request_result* res);

/* ------------------------------------------------------- measurement kernels */

/* Read `bytes` (multiple of 16) and write one partial checksum per workgroup
 * to d_partial (tq_read_peak_scratch_bytes() bytes): the streaming-read
 * ceiling of the device. */
size_t tq_read_peak_scratch_bytes(void);
tq_status tq_read_peak(const void* d_src, size_t bytes, int64_t* d_partial, hipStream_t stream);
/* Write `bytes` (multiple of 16) of a pattern; used to evict caches between timed repetitions. */
tq_status tq_fill(void* d_dst, size_t bytes, uint32_t pattern, hipStream_t stream);

/* ------------------------------------------------------------ Parquet scan */

/* Scan-side decode of Parquet files (Section 3.3.3, Byte Range Pre-loading:
 * the file's metadata gives the exact byte ranges a scan needs, close ranges
 * are merged into one read, and the bytes land in pool pages ahead of the
 * compute task, which is left with decoding; Section 4 reads Parquet inputs).
 * Supported: flat schemas; INT32 and INT64 columns, required or optional;
 * data pages v1 and v2 in PLAIN or dictionary encoding (RLE_DICTIONARY /
 * PLAIN_DICTIONARY, dictionary pages PLAIN); column chunks uncompressed or
 * Snappy-compressed (inflated on the GPU).
 * Other codecs, encodings, types and nested columns are rejected with
 * TQ_EINVAL when the file is opened or the preload is planned. */
typedef struct tq_parquet tq_parquet;
typedef struct tq_preload tq_preload;

/* Open a file and read its footer (host). The handle owns the file
 * descriptor; tq_parquet_close releases both. */
tq_status tq_parquet_open(const char* path, tq_parquet** out);
void tq_parquet_close(tq_parquet* pq);
int64_t tq_parquet_num_rows(const tq_parquet* pq);
int32_t tq_parquet_num_row_groups(const tq_parquet* pq);
int64_t tq_parquet_row_group_rows(const tq_parquet* pq, int32_t rg);
int32_t tq_parquet_num_columns(const tq_parquet* pq);
/* Column c: its name (owned by the handle), output type (TQ_I32 / TQ_I64, 0
 * if not decodable) and whether it may hold NULLs (an optional column). */
tq_status tq_parquet_column(const tq_parquet* pq, int32_t c, const char** name, int32_t* type, int32_t* nullable);
/* The byte range of column c's chunk in row group rg, and its codec. */
tq_status tq_parquet_chunk(const tq_parquet* pq, int32_t rg, int32_t c, int64_t* file_off, int64_t* bytes,
                           int32_t* codec);

/* Byte Range Pre-loading: the chunks of columns h_cols[0..ncol) in row
 * groups [rg0, rg1), sorted by offset, ranges at most merge_gap bytes apart
 * merged into one read; pool pages are taken for every read (TQ_ENOMEM if the
 * pool has too few) and up to four host threads start reading into them,
 * each taking the next piece of at most 2 MiB within one page; the call
 * returns at once. The file handle and the pool must outlive the preload
 * (tq_preload_free waits for the reads). */
tq_status tq_parquet_preload(tq_parquet* pq, tq_pagepool* pool, int32_t rg0, int32_t rg1, const int32_t* h_cols,
                             int32_t ncol, int64_t merge_gap, tq_preload** out);
int32_t tq_preload_num_reads(const tq_preload* p);
tq_status tq_preload_read(const tq_preload* p, int32_t i, int64_t* file_off, int64_t* bytes);
int64_t tq_preload_rows(const tq_preload* p); /* rows of the row groups */
/* Waits for the reads, walks the page headers (host) and returns the device
 * work bytes tq_parquet_decode needs. */
tq_status tq_preload_work_bytes(tq_preload* p, size_t* bytes);
/* After tq_preload_work_bytes: the pages found, in file order (kind 0 data,
 * 2 dictionary; encoding 0 PLAIN, 8 dictionary indices). */
int64_t tq_preload_num_pages(const tq_preload* p);
tq_status tq_preload_page(const tq_preload* p, int64_t i, int64_t* row0, int32_t* nrows, int32_t* col, int32_t* kind,
                          int32_t* encoding);
/* Decode into out[c] (c over the preload's columns): out[c].type = the
 * column's type, out[c].data holds tq_preload_rows() values, out[c].valid a
 * bitmap of as many bits, written as whole 32-bit words: it must hold
 * ((rows + 31) / 32) * 4 bytes, 4-byte aligned (required for a nullable
 * column, optional otherwise: all ones then). NULL rows get value 0. The bytes are copied from
 * the pool pages into d_work (256-byte aligned, tq_preload_work_bytes bytes)
 * and decoded there by kernels on `stream`; the call returns once the copies
 * are done and the pages are back in the pool, with the kernels enqueued.
 * Errors found by the kernels (a malformed stream, a dictionary index out of
 * range) are latched in d_work: tq_check(d_work, stream) reports them. A
 * preload is decoded once (a second call returns TQ_EINVAL). */
tq_status tq_parquet_decode(tq_preload* p, void* d_work, size_t work_bytes, const tq_col* out, hipStream_t stream);
/* Waits for the reads, returns unused pages to the pool and frees the handle. */
void tq_preload_free(tq_preload* p);

#ifdef __cplusplus
}
#endif
#endif /* TQ_H */
