// Parquet scan, device side: decodes the pages of preloaded column chunks
// into Arrow columns (values + validity bitmap). Section 3.3.3 leaves the
// compute task only decompression and decoding once the byte ranges are in
// memory; these kernels are that work, for INT32 / INT64 pages in PLAIN or
// dictionary (RLE_DICTIONARY) encoding, flat columns, required or optional
// (definition levels), uncompressed or Snappy-compressed.
//
// The definition levels and the dictionary indices are RLE/bit-packed hybrid
// streams, whose runs can only be found one after another. So:
//   k_pq_snappy inflates each compressed page body (one wave per page);
//   k_pq_span   finds each page's level and value sections;
//   k_pq_dict   copies each dictionary page's values to an aligned array;
//   k_pq_walk   one wave per (page, stream) walks the run headers out of an
//               LDS window of the stream (one lane; the wave stages the bytes)
//               and writes a run table, plus a checkpoint every kPqTile items
//               (the run holding that item, and the present rows before it);
//   k_pq_decode one workgroup per kPqTile rows of a page: from its checkpoint
//               it stages the tile's runs in LDS, finds each row's level and
//               value index (a workgroup scan of the present rows), decodes
//               the value (PLAIN, or dictionary index then gather) and writes
//               the values and the validity bits.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "parquet.h"

namespace tq {

constexpr int kWalkWin = 16384;  // bytes of a stream staged in LDS at a time
constexpr int kDecBlock = 256;
constexpr int kDecRows = kPqTile / kDecBlock;  // rows per thread
constexpr int kTileRuns = 1024 + 1;           // runs of a tile's rows (each run holds at least one item)

struct PqHeader {
  uint32_t magic;
  int32_t err;
};

__device__ __forceinline__ void pq_error(PqHeader* h, int32_t code) { atomicCAS(&h->err, 0, code); }

// Little-endian bytes [p, p + width) of the raw area (width 4 or 8), from
// aligned 32-bit loads; may read up to 8 bytes past the value (the raw area
// is padded).
__device__ __forceinline__ uint64_t ld_le(const uint8_t* raw, int64_t p, int width) {
  const uint32_t* a = reinterpret_cast<const uint32_t*>(raw + (p & ~(int64_t)3));
  const uint32_t sh = (uint32_t)(p & 3) * 8;
  const uint32_t w0 = a[0], w1 = a[1];
  const uint32_t lo = sh ? (w0 >> sh) | (w1 << (32 - sh)) : w0;
  if (width == 4) return lo;
  const uint32_t w2 = a[2];
  const uint32_t hi = sh ? (w1 >> sh) | (w2 << (32 - sh)) : w1;
  return (uint64_t)hi << 32 | lo;
}

__global__ void k_pq_init(PqHeader* h) {
  h->magic = kScanMagic;
  h->err = 0;
}

__global__ void k_pq_zero(uint32_t* words, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    words[i] = 0u;
}

// ------------------------------------------------------------------ Snappy
//
// The format (Snappy's raw block: the uncompressed length as a varint, then
// elements: a literal of n bytes that follow its tag, or a copy of n bytes
// from `offset` bytes back in the output, which may overlap what it writes)
// is sequential: an element's start is known only from the one before. Three
// passes: k_pq_snappy_scan finds the chain of every body (a workgroup per
// body; in each step each thread decodes the element that would start at its
// byte, and the real chain is picked out by pointer doubling) and where each
// 64 KiB output fragment's first element starts; k_pq_snappy_frag inflates
// the fragments independently, one wave each in LDS, when no element crosses
// a fragment or copies from before its own (what the reference compressor
// writes, compressing 64 KiB at a time); k_pq_snappy inflates any other body
// with one wave in order, through a 64 KiB LDS ring holding the last 64 KiB
// written, 8 KiB at a time to the device buffer.
constexpr int kRing = 65536;
constexpr int kFlushBytes = 8192;
constexpr int kInWin = 16384;

__device__ __forceinline__ uint32_t in_byte(const uint32_t* w, int32_t i) { return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu; }

// The Snappy element that would start at window byte i: the input bytes it
// takes (tag, length or offset bytes, literal payload), the output bytes it
// writes, and its copy offset (0 for a literal; -1 if 0 or impossibly far).
__device__ __forceinline__ void snappy_candidate(const uint32_t* win, int32_t i, int32_t& c_adv, int32_t& c_len,
                                                 int32_t& c_off) {
  uint32_t cb[5];
#pragma unroll
  for (int k = 0; k < 5; k++) cb[k] = in_byte(win, i + k);
  const uint32_t t = cb[0];
  if ((t & 3) == 0) {
    const uint32_t l6 = t >> 2;
    uint32_t lit = l6 + 1, hb = 1;
    if (l6 >= 60) {
      const int nb = (int)l6 - 59;
      uint32_t v = 0;
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (k < nb) v |= cb[1 + k] << (8 * k);
      lit = v >= (1u << 30) ? (1u << 30) : v + 1;  // too long for any page: caught by the caller
      hb = 1 + nb;
    }
    c_adv = (int32_t)(hb + lit);
    c_len = (int32_t)lit;
    c_off = 0;
  } else if ((t & 3) == 1) {
    c_adv = 2;
    c_len = 4 + (int32_t)((t >> 2) & 7);
    c_off = (int32_t)(((t >> 5) << 8) | cb[1]);
  } else if ((t & 3) == 2) {
    c_adv = 3;
    c_len = (int32_t)(t >> 2) + 1;
    c_off = (int32_t)(cb[1] | cb[2] << 8);
  } else {
    c_adv = 5;
    c_len = (int32_t)(t >> 2) + 1;
    const uint32_t o = cb[1] | cb[2] << 8 | cb[3] << 16 | cb[4] << 24;
    c_off = o >= (1u << 30) ? -1 : (int32_t)o;
  }
  if ((t & 3) != 0 && c_off == 0) c_off = -1;  // c_off == 0 marks a literal and nothing else
}

// An LDS window of a compressed body: input bytes [wbase, wbase + WIN),
// loaded as aligned dwords of the raw area (wbase may be up to 3 bytes
// before 0). ensure() is called alike by every lane of the wave.
template <int WIN>
struct InWindowT {
  uint32_t* win;
  const uint8_t* raw;
  int64_t c_off;
  int32_t in_len;
  int32_t wbase;
  // NT: the threads that load (the workgroup, or one wave of it: then kSync
  // false, and only that wave reads the window)
  template <int NT = 64, bool kSync = true>
  __device__ void ensure(int32_t at, int32_t need) {
    if (at >= wbase && at + need <= wbase + WIN) return;
    // 16-byte loads, all issued before any is stored: one memory round trip
    const int64_t abs0 = (c_off + at) & ~(int64_t)15;
    wbase = (int32_t)(abs0 - c_off);
    constexpr int kV = (WIN / 16 + 1 + NT - 1) / NT;  // loads per thread
    v4i32 t[kV];
#pragma unroll
    for (int u = 0; u < kV; u++) {
      const int i = (int)threadIdx.x + NT * u;
      const int64_t a = abs0 + 16 * (int64_t)i;  // a load starting before the input's end stays in the padded area
      t[u] = i < WIN / 16 + 1 && a < c_off + in_len ? *reinterpret_cast<const v4i32*>(raw + a) : v4i32{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < kV; u++) {
      const int i = (int)threadIdx.x + NT * u;
      if (i < WIN / 16 + 1) reinterpret_cast<v4i32*>(win)[i] = t[u];
    }
    if (kSync)
      __syncthreads();
    else
      asm volatile("" ::: "memory");  // one wave's LDS accesses take effect in program order
  }
  __device__ uint32_t byte(int32_t at) const { return in_byte(win, at - wbase); }
};
using InWindow = InWindowT<kInWin>;

// The length preamble (a varint) of a Snappy body; its size in *ip, false
// if malformed.
template <int NT = 64>
__device__ bool snappy_preamble(InWindow& w, uint32_t* ulen, int32_t* ip) {
  w.ensure<NT>(0, 8);
  uint32_t v = 0;
  int32_t i = 0;
  for (int sh = 0;; sh += 7) {
    const uint32_t b = i < w.in_len ? w.byte(i) : 0x80u;
    i++;
    v |= (b & 0x7f) << sh;
    if (!(b & 0x80)) break;
    if (sh >= 28 || i >= w.in_len) return false;
  }
  *ulen = v;
  *ip = i;
  return true;
}

constexpr int kFrag = 65536;  // the reference compressor's independent fragments
// Every element takes at least two input bytes (a tag and a literal byte, or a
// copy's tag and offset), so a chain crosses 64 bytes in at most 32 hops: five
// doubling (or lifting) steps of 2^k hops cover it.
constexpr int kHops = 5;

// Pass 1, one workgroup of kScanWaves waves per compressed body: follows the
// element chain, records where each 64 KiB output fragment's first element
// starts, and flags the body when an element crosses a fragment or copies
// from before its fragment (then the body is inflated by one wave, in order,
// with every access checked). flags: 0 fragments independent, 1 inflate in
// order, 2 malformed.
//
// The body is taken in blocks of kScanBlk input bytes, 64 per sub-batch, one
// sub-batch per wave of waves 1 .. kScanWaves - 1, each thread decoding the
// element that would start at its byte. (1) Each wave builds, by pointer
// doubling, the start 2^k elements on from each lane and the output bytes of
// those 2^k elements (k < kHops), up to where the chain leaves the sub-batch.
// (2) Wave 0 walks the chain through the block a sub-batch per hop (register
// reads of the sub-batches' exits), giving each sub-batch the lane its
// elements start at and the output position there. (3) Each lane, from its
// sub-batch's first element, jumps 2^k elements (k = kHops - 1 .. 0) while that
// lands at or before it: it is an element if it lands on itself, and the
// jumps' output bytes give its output position. The three run as a pipeline
// with one pair of barriers per block: while wave 0 walks block i, the other
// waves build block i + 1's tables and mark block i - 1's elements. A block
// starts where the one before it ends, or where the chain is when a literal
// has skipped a whole block. (A register walk per element in (3), in place of
// the jumps, took 1.7x as long.)
constexpr int kScanWaves = 16;
constexpr int kScanSub = kScanWaves - 1;   // sub-batches per block
constexpr int kScanBlk = 64 * kScanSub;    // input bytes per block
// element lengths are summed in 32 bits clamped to this; a body with a longer
// element is flagged for the in-order pass
constexpr int32_t kLenClamp = 1 << 24;

// A lane's doubling tables for one block (phase 1, kept for phase 3).
struct ScanTab {
  int32_t jk[kHops];   // the start 2^k elements on, sub-batch-relative (>= 64: past it)
  uint32_t sk[kHops];  // the output bytes of those 2^k elements
  int32_t len, off;
};

__global__ __launch_bounds__(64 * kScanWaves) void k_pq_snappy_scan(const PqPage* pages, const int32_t* cpages,
                                                                    const uint8_t* raw, int32_t* frag_in,
                                                                    int32_t* flags, PqHeader* hdr) {
  __shared__ __align__(16) uint32_t wbuf[kInWin / 4 + 4];
  __shared__ int2 exs[2][kScanBlk];      // where the chain from each byte leaves its sub-batch
                                         // (block-relative), and the output bytes up to there
  __shared__ int32_t ent[2][kScanSub];   // each sub-batch's first element (lane; -1: none)
  __shared__ int64_t qent[2][kScanSub];  // and its output position
  __shared__ uint32_t s_end[2];          // the first element at or past the output's end:
                                         // position << 1 | malformed (per iteration parity)
  __shared__ int64_t s_pos;              // the walker's place in the chain after its block
  __shared__ int32_t s_dep, s_bad;
  const PqPage pg = pages[cpages[blockIdx.x]];
  InWindow w{wbuf, raw, pg.c_off, (int32_t)pg.c_len, INT32_MIN / 2};
  const int64_t out_len = pg.u_len;
  int32_t* fi = frag_in + pg.frag0;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63, sb = wv - 1;
  uint32_t ulen;
  int32_t ip0;
  bool bad = !snappy_preamble<64 * kScanWaves>(w, &ulen, &ip0) || ulen != (uint32_t)out_len;
  if (t == 0) {
    s_dep = 0;
    s_bad = 0;
    s_end[0] = s_end[1] = UINT32_MAX;
    s_pos = ip0;
  }
  // (1) for the block at bs, into exs[par] and T (waves 1 ..)
  auto tables = [&](int64_t bs, int par, ScanTab& T) {
    int32_t c_adv, c_len, c_off;
    snappy_candidate(w.win, (int32_t)(bs - w.wbase) + 64 * sb + lane, c_adv, c_len, c_off);
    T.len = c_len;
    T.off = c_off;
    int32_t J = lane + c_adv;
    uint32_t S = (uint32_t)min(c_len, kLenClamp);
#pragma unroll
    for (int k = 0; k < kHops; k++) {
      T.jk[k] = J;
      T.sk[k] = S;
      const int src = J < 64 ? J : lane;
      const int32_t Jn = __shfl(J, src);
      const uint32_t Sn = __shfl(S, src);
      if (J < 64) {
        J = Jn;
        S += Sn;
      }
    }
    exs[par][64 * sb + lane] = make_int2(64 * sb + J, (int32_t)S);  // S <= 64 * kLenClamp
  };
  // (3) for the block at bs (walked into ent[par]), iteration parity ipar
  auto mark = [&](int64_t bs, int par, int ipar, const ScanTab& T) {
    const int32_t e = ent[par][sb];
    int32_t pos = e < 0 ? 0 : e;
    uint32_t acc = 0;
#pragma unroll
    for (int k = kHops - 1; k >= 0; k--) {
      const int32_t c = __shfl(T.jk[k], pos);
      const uint32_t a = __shfl(T.sk[k], pos);
      if (c <= lane) {
        pos = c;
        acc += a;
      }
    }
    const bool el = e >= 0 && e <= lane && pos == lane;
    const int64_t qs = (e >= 0 ? qent[par][sb] : 0) + (int64_t)acc;  // an element's first output byte
    const int64_t at = bs + 64 * sb + lane;                          // and its first input byte
    // the chain's end: its first element at or past the output's end, which
    // must start at the input's end exactly at the output's end
    const uint64_t endm = __ballot(el && qs >= out_len);
    if (endm && lane == __builtin_ctzll(endm))
      atomicMin(&s_end[ipar], (uint32_t)at << 1 | (uint32_t)(at != w.in_len || qs != out_len));
    if (el && qs < out_len) {
      const int64_t fs = qs & ~(int64_t)(kFrag - 1);
      if (qs == fs) fi[qs >> 16] = (int32_t)at;
      if (T.len > kLenClamp || qs + T.len > fs + kFrag || (T.off != 0 && (T.off < 0 || qs - T.off < fs)))
        s_dep = 1;
    }
  };
  // (2) the walker, wave 0: the chain through the block at bs (tables
  // exs[par]). The wave holds the block's exits in registers (lane l of ex[s]:
  // sub-batch s's byte l) and hops with register reads only, sub-batch by
  // sub-batch; lane s then stores sub-batch s's entry.
  int64_t wpos = ip0, wq = 0;  // (wave 0) the chain's next element and its output position
  bool wstop = false;          // (wave 0) the sub-batch of the chain's end is recorded
  auto walk = [&](int64_t bs, int par) {
    int2 ex[kScanSub];
#pragma unroll
    for (int s = 0; s < kScanSub; s++) ex[s] = exs[par][64 * s + lane];
    int32_t my_ent = -1;
    int64_t my_q = 0;
    int64_t rel = wstop ? (int64_t)kScanBlk : wpos - bs;  // >= 0: a block starts at or before the chain's place
#pragma unroll
    for (int s = 0; s < kScanSub; s++) {
      if (!wstop && (rel >> 6) == s) {  // (uniform)
        const int l = (int)(rel & 63);
        if (lane == s) {
          my_ent = l;
          my_q = wq;
        }
        if (wq >= out_len) {
          wstop = true;  // this sub-batch holds the chain's end (phase 3 finds it)
        } else {
          wq += __builtin_amdgcn_readlane(ex[s].y, l);
          rel = __builtin_amdgcn_readlane(ex[s].x, l);
        }
      }
    }
    if (lane < kScanSub) {
      ent[par][lane] = my_ent;
      qent[par][lane] = my_q;
    }
    if (!wstop) {
      wpos = bs + rel;
      // the chain left the input short of the output's end
      if (lane == 0 && wpos > w.in_len && wq < out_len) s_bad = 1;
    }
    if (lane == 0) s_pos = wpos;
  };

  ScanTab A, B, C;  // the tables of blocks i - 1, i, i + 1
  bool dep = false, done = bad;
  int64_t b_prev = 0, b_cur = ip0, entry = ip0;
  __syncthreads();
  if (!done) {
    w.ensure<64 * kScanWaves>(b_cur, kScanBlk + 8);
    if (wv > 0) tables(b_cur, 0, B);
  }
  __syncthreads();
  // every thread holds the same block starts and `done`: the loop is uniform
  for (int64_t i = 0; !done; i++) {
    // block i + 1 starts after block i, or where the chain is if it is past
    // block i already (a literal skipped it)
    const int64_t b_next = entry > b_cur + kScanBlk ? entry : b_cur + kScanBlk;
    w.ensure<64 * kScanWaves>(b_next, kScanBlk + 8);
    const int par = (int)(i & 1);
    if (wv > 0) {
      if (i > 0) mark(b_prev, par ^ 1, par, A);
      tables(b_next, par ^ 1, C);
    } else {
      walk(b_cur, par);
      if (lane == 0) s_end[par ^ 1] = UINT32_MAX;  // for the next iteration's marks
    }
    __syncthreads();
    // the shared state is read between two barriers: no thread writes it
    // again before every thread has read it
    const uint32_t end = s_end[par];
    entry = s_pos;
    if (s_dep != 0) {
      dep = true;
      done = true;
    } else if (end != UINT32_MAX) {
      done = true;
      bad = (end & 1) != 0;
    } else if (s_bad != 0) {
      bad = true;
      done = true;
    }
    __syncthreads();
    A = B;
    B = C;
    b_prev = b_cur;
    b_cur = b_next;
  }
  if (t == 0) {
    flags[blockIdx.x] = dep ? 1 : bad ? 2 : 0;
    if (bad && !dep) pq_error(hdr, TQ_EINVAL);
  }
}

// Pass 2, one workgroup of two waves per 64 KiB fragment of a body whose
// fragments are independent, inflated into an LDS copy of the fragment that is
// then written out. Wave 0 parses. A batch: lane i decodes the element that
// would start at input byte ip + i; doubling and lifting (as in the scan, from
// lane 0) give the elements and their output positions. Wave 0 stores the
// literal payload bytes (those among the batch's 64 input bytes by the lanes
// holding them, the payload of a literal running past them by the whole wave)
// and queues the batch's copies; wave 1 runs the copies, which read earlier
// output, in order. They work in rounds: wave 0 parses up to kFragQ batches
// into one half of the queue while wave 1 runs the copies the other half took
// in the round before; a barrier ends each round and makes its literal bytes
// visible to the copies of the next. A wave's LDS accesses take effect in
// program order, so between copies only the compiler is fenced.
constexpr int kFragWin = 8192;  // (64 KiB fragment + this window + the queue: two workgroups per CU)
constexpr int kFragQ = 4;       // batches per round

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

__global__ __launch_bounds__(2 * kWave) void k_pq_snappy_frag(const PqPage* pages, const int32_t* cpages,
                                                              const int32_t* frag_cpage, uint8_t* raw,
                                                              const int32_t* frag_in, const int32_t* flags,
                                                              PqHeader* hdr) {
  __shared__ uint32_t buf[kFrag / 4];
  __shared__ __align__(16) uint32_t wbuf[kFragWin / 4 + 4];
  __shared__ uint2 cq[2][kFragQ][kWave];  // a queued batch, per lane: output offset | length << 16, copy offset
  __shared__ uint64_t cmask[2][kFragQ];   // the lanes of its copies
  __shared__ int32_t s_nb[2], s_done, s_bad;
  uint8_t* fb = reinterpret_cast<uint8_t*>(buf);
  const int32_t ci = frag_cpage[blockIdx.x];
  if (flags[ci] != 0) return;
  const PqPage pg = pages[cpages[ci]];
  const int32_t f = (int32_t)(blockIdx.x - pg.frag0);
  const int32_t out_len = (int32_t)pg.u_len;
  const int32_t fs = f * kFrag, fe = min(fs + kFrag, out_len);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (threadIdx.x == 0) {
    s_nb[0] = s_nb[1] = 0;
    s_done = s_bad = 0;
  }
  __syncthreads();
  InWindowT<kFragWin> w{wbuf, raw, pg.c_off, (int32_t)pg.c_len, INT32_MIN / 2};  // wave 0's
  const uint8_t* in = raw + pg.c_off;
  int32_t ip = frag_in[pg.frag0 + f], q = fs;
  bool parsed = false, failed = false;  // the same in every thread
  for (int r = 0;; r++) {
    const int par = r & 1;
    if (wave == 0 && !parsed) {
      int nb = 0;
      bool bad = ip < 0 || ip >= w.in_len;
      while (!bad && nb < kFragQ && q < fe) {
        w.template ensure<kWave, false>(ip, 64 + 8);
        int32_t c_adv, c_len, c_off;
        const int32_t wi = ip + lane - w.wbase;
        snappy_candidate(w.win, wi, c_adv, c_len, c_off);
        const uint32_t mine = in_byte(w.win, wi);  // input byte ip + lane
        int32_t jk[kHops];
        uint32_t sk[kHops];
        int32_t J = lane + c_adv;
        uint32_t S = (uint32_t)min(c_len, kLenClamp);
#pragma unroll
        for (int k = 0; k < kHops; k++) {
          jk[k] = J;
          sk[k] = S;
          const int src = J < 64 ? J : lane;
          const int32_t Jn = __shfl(J, src);
          const uint32_t Sn = __shfl(S, src);
          if (J < 64) {
            J = Jn;
            S += Sn;
          }
        }
        int32_t pos = 0;
        uint32_t acc = 0;
#pragma unroll
        for (int k = kHops - 1; k >= 0; k--) {
          const int32_t c = __shfl(jk[k], pos);
          const uint32_t a = __shfl(sk[k], pos);
          if (c <= lane) {
            pos = c;
            acc += a;
          }
        }
        const int64_t qs = (int64_t)q + acc;  // an element's first output byte
        const uint64_t live = __ballot(pos == lane && qs < fe);  // the fragment's elements in the batch (lane 0: q < fe)
        const bool me = (live >> lane) & 1;
        const int32_t at = ip + lane;
        // the scan checked the chain; these checks keep every access in bounds
        // regardless (a length past the fragment also catches a clamped one)
        const bool badl = me && (at >= w.in_len || c_len > fe - qs || c_adv > w.in_len - at ||
                                 (c_off != 0 && (c_off <= 0 || c_off > qs - fs)));
        if (__ballot(badl)) {
          bad = true;
          break;
        }
        const int32_t lq = (int32_t)(qs - fs);  // (live lanes) its offset in the fragment, below 2^16
        // literal payload bytes among the batch's input bytes: lane j's byte
        // belongs to the last element starting at or before j
        const int eo = 63 - __builtin_clzll(live & ((2ull << lane) - 1));
        const int32_t e_len = __shfl(c_len, eo), e_adv = __shfl(c_adv, eo), e_off = __shfl(c_off, eo);
        const int32_t e_lq = __shfl(lq, eo);
        const int32_t rel = lane - (eo + e_adv - e_len);  // its place in that element's payload
        if (e_off == 0 && rel >= 0 && rel < e_len) fb[e_lq + rel] = (uint8_t)mine;
        // the batch's last element: a literal may run past the batch's input bytes
        const int L = 63 - __builtin_clzll(live);
        const int32_t l_len = __builtin_amdgcn_readlane(c_len, L), l_adv = __builtin_amdgcn_readlane(c_adv, L);
        const int32_t l_off = __builtin_amdgcn_readlane(c_off, L), l_lq = __builtin_amdgcn_readlane(lq, L);
        if (l_off == 0 && L + l_adv > 64) {
          const int32_t p0 = L + l_adv - l_len;  // payload start, batch-relative
          const int32_t src = ip + p0;
          const bool in_win = src >= w.wbase && src + l_len <= w.wbase + kFragWin;
          for (int32_t j = max(0, 64 - p0) + lane; j < l_len; j += 64)
            fb[l_lq + j] = in_win ? (uint8_t)w.byte(src + j) : in[src + j];
        }
        // the copies (at most 64 bytes each) go to the queue
        const uint64_t copies = live & __ballot(c_off != 0);
        cq[par][nb][lane] = make_uint2(((uint32_t)lq & 0xffffu) | ((uint32_t)c_len << 16), (uint32_t)c_off);
        if (lane == 0) cmask[par][nb] = copies;
        nb++;
        q = fs + l_lq + l_len;
        ip += L + l_adv;
      }
      if (lane == 0) {
        s_nb[par] = nb;
        if (bad) s_bad = 1;
        if (!bad && q >= fe) s_done = 1;
      }
    } else if (wave == 1 && r > 0) {
      // the copies queued in the round before, in order
      const int cp = par ^ 1;
      const int nb = s_nb[cp];
      for (int b = 0; b < nb; b++) {
        uint64_t rest = cmask[cp][b];
        const uint2 e = cq[cp][b][lane];
        while (rest) {
          const int l = __builtin_ctzll(rest);
          rest &= rest - 1;
          const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)e.x, l);
          const int32_t off = __builtin_amdgcn_readlane((int)e.y, l);
          const int32_t dq = (int32_t)(x & 0xffffu), len = (int32_t)(x >> 16);
          if (lane < len) fb[dq + lane] = fb[dq - off + (off >= len ? lane : lane % off)];
          compiler_fence();
        }
      }
    }
    __syncthreads();
    const bool done = s_done != 0, bad = s_bad != 0;  // read between two barriers: written only before the first
    __syncthreads();
    if (bad) {
      failed = true;
      break;
    }
    if (parsed) break;  // this round ran the last queued copies
    parsed = done;
  }
  if (failed) {
    if (threadIdx.x == 0) pq_error(hdr, TQ_EINVAL);
    return;
  }
  uint32_t* dst = reinterpret_cast<uint32_t*>(raw + pg.u_off + fs);  // 256-aligned, padded past the body
  for (int i = threadIdx.x; i < ((fe - fs + 3) >> 2); i += 2 * kWave) dst[i] = buf[i];
}

// A body the scan flagged (1), inflated by one wave in order through a 64 KiB
// ring of the latest output.
__global__ __launch_bounds__(64) void k_pq_snappy(const PqPage* pages, const int32_t* cpages, uint8_t* raw,
                                                  const int32_t* flags, PqHeader* hdr) {
  __shared__ uint32_t ring[kRing / 4];
  __shared__ uint32_t win[kInWin / 4 + 4];
  uint8_t* rb = reinterpret_cast<uint8_t*>(ring);
  if (flags[blockIdx.x] != 1) return;
  const PqPage pg = pages[cpages[blockIdx.x]];
  const uint8_t* in = raw + pg.c_off;
  // page bodies are at most 1 GiB (checked on the host): 32-bit positions
  const int32_t in_len = (int32_t)pg.c_len, out_len = (int32_t)pg.u_len;
  uint8_t* out = raw + pg.u_off;
  const int lane = threadIdx.x;
  // the input window holds input bytes [wbase, wbase + kInWin), loaded as
  // aligned dwords of the raw area (wbase may be up to 3 bytes before 0)
  int32_t wbase = INT32_MIN / 2;
  auto window = [&](int32_t at, int32_t need) {  // uniform: every lane asks for the same bytes
    if (at >= wbase && at + need <= wbase + kInWin) return;
    const int64_t abs0 = (pg.c_off + at) & ~(int64_t)3;
    wbase = (int32_t)(abs0 - pg.c_off);
    for (int i = lane; i < kInWin / 4 + 4; i += 64) {
      const int64_t a = abs0 + 4 * (int64_t)i;  // a dword starting before the input's end stays in the padded area
      win[i] = a < pg.c_off + in_len ? *reinterpret_cast<const uint32_t*>(raw + a) : 0u;
    }
    __syncthreads();
  };
  bool bad = false;
  // the uncompressed length
  window(0, 8);
  uint32_t ulen = 0;
  int32_t ip = 0;
  for (int sh = 0;; sh += 7) {
    const uint32_t b = ip < in_len ? in_byte(win, ip - wbase) : 0x80u;
    ip++;
    ulen |= (b & 0x7f) << sh;
    if (!(b & 0x80)) break;
    if (sh >= 28 || ip >= in_len) {
      bad = true;
      break;
    }
  }
  if (ulen != (uint32_t)out_len) bad = true;
  int32_t q = 0, flushed = 0;
  // writes the ring's final bytes out in whole chunks below `upto` (a chunk
  // boundary), or everything left once upto is the output's end
  auto flush_to = [&](int32_t upto) {
    while (flushed + kFlushBytes <= upto || (upto == out_len && flushed < out_len)) {
      const int32_t n = min(kFlushBytes, out_len - flushed);
      uint32_t* dst = reinterpret_cast<uint32_t*>(out + flushed);  // the output area is 256-aligned and padded
      const int base = (flushed & (kRing - 1)) >> 2;
      for (int i = lane; i < ((n + 3) >> 2); i += 64) dst[i] = ring[base + i];
      flushed += n;
    }
  };
  while (!bad && q < out_len) {
    // Parse a batch: lane i decodes the element that would start at input
    // byte ip + i; the chain of real elements is then followed from lane 0
    // with register reads (the element after the one at lane r is at lane
    // r + its byte length), and each element is executed as it is reached.
    window(ip, 64 + 8);
    int32_t c_adv, c_len, c_off;  // bytes the element takes, bytes it writes, copy offset (0: a literal)
    snappy_candidate(win, ip + lane - wbase, c_adv, c_len, c_off);
    int32_t rel = 0;
    while (rel < 64 && !bad && q < out_len) {
      const int32_t at = ip + rel;
      if (at >= in_len) {
        bad = true;
        break;
      }
      const int32_t adv = __builtin_amdgcn_readlane(c_adv, rel);
      const int32_t len = __builtin_amdgcn_readlane(c_len, rel);
      const int32_t off = __builtin_amdgcn_readlane(c_off, rel);
      const bool literal = off == 0;
      const int32_t src = at + adv - len;                        // a literal's first payload byte
      if (len > out_len - q || adv > in_len - at || (!literal && (off <= 0 || off > q))) {
        bad = true;
        break;
      }
      if (literal) {
        // from the window when the payload lies in it, else straight from memory
        const bool in_win = src >= wbase && src + len <= wbase + kInWin;
        for (int32_t s0 = 0; s0 < len; s0 += kFlushBytes) {
          const int32_t pl = min(kFlushBytes, len - s0);
          const int32_t need = q + s0 + pl - kRing;  // ring slots about to be reused: those bytes are final
          if (need > flushed) flush_to(((need + kFlushBytes - 1) / kFlushBytes) * kFlushBytes);
          for (int32_t j = s0 + lane; j < s0 + pl; j += 64) {
            const uint8_t b = in_win ? (uint8_t)in_byte(win, src + j - wbase) : in[src + j];
            rb[(q + j) & (kRing - 1)] = b;
          }
        }
      } else {
        // a copy is at most 64 bytes; its sources lie below q (final; in the
        // ring when less than 64 KiB back)
        const int32_t need = q + len - kRing;
        if (need > flushed) flush_to(((need + kFlushBytes - 1) / kFlushBytes) * kFlushBytes);
        const bool far = off >= kRing;
        if (far) {
          flush_to(q & ~(kFlushBytes - 1));  // every source byte lies below (q - off + 64 < q - 8 KiB)
          __threadfence();                   // those stores are visible before the loads below
        }
        if (lane < len) {
          const int32_t sp = q - off + (off >= len ? lane : lane % off);
          const uint8_t b = far ? out[sp] : rb[sp & (kRing - 1)];
          rb[(q + lane) & (kRing - 1)] = b;
        }
      }
      q += len;
      rel += adv;
    }
    ip += rel;
  }
  if (!bad) flush_to(out_len);
  if (bad && lane == 0) pq_error(hdr, TQ_EINVAL);
}

// The level and value sections of every page, once bodies are inflated.
__global__ void k_pq_span(const PqPage* pages, int npages, const uint8_t* raw, PqSpan* spans, PqHeader* hdr) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npages; i += gridDim.x * blockDim.x) {
    const PqPage pg = pages[i];
    PqSpan sp{pg.def_off, pg.def_end, pg.val_off, pg.val_end};
    if (pg.def_off == kPqLevelsInBody) {
      if (pg.val_off + 4 > pg.val_end) {
        pq_error(hdr, TQ_EINVAL);
        sp = PqSpan{-1, -1, pg.val_end, pg.val_end};
      } else {
        const int64_t len = (int64_t)(uint32_t)ld_le(raw, pg.val_off, 4);
        if (pg.val_off + 4 + len > pg.val_end) {
          pq_error(hdr, TQ_EINVAL);
          sp = PqSpan{pg.val_off + 4, pg.val_off + 4, pg.val_end, pg.val_end};
        } else {
          sp = PqSpan{pg.val_off + 4, pg.val_off + 4 + len, pg.val_off + 4 + len, pg.val_end};
        }
      }
    }
    spans[i] = sp;
  }
}

constexpr int kDictBlocks = 16;  // workgroups per dictionary page

// kDictBlocks workgroups per dictionary page.
__global__ __launch_bounds__(kDecBlock) void k_pq_dict(const PqPage* pages, const int32_t* dict_pages,
                                                       const uint8_t* raw, uint8_t* dict) {
  const PqPage pg = pages[dict_pages[blockIdx.x / kDictBlocks]];
  const int w = pg.width;
  uint8_t* out = dict + pg.dict_off;
  const int part = blockIdx.x % kDictBlocks;
  for (int64_t e = (int64_t)part * kDecBlock + threadIdx.x; e < pg.dict_n; e += (int64_t)kDictBlocks * kDecBlock) {
    const uint64_t v = ld_le(raw, pg.val_off + e * w, w);
    if (w == 8) reinterpret_cast<uint64_t*>(out)[e] = v;
    else reinterpret_cast<uint32_t*>(out)[e] = (uint32_t)v;
  }
}

__device__ __forceinline__ uint32_t win_byte(const uint32_t* win, int64_t i) { return (win[i >> 2] >> ((i & 3) * 8)) & 0xffu; }

// Items equal to 1 among the first n of a bit-packed run of bit width 1 at
// raw byte `at` (window bytes when they are staged there).
__device__ uint32_t ones_prefix(const uint32_t* win, int64_t wbase, int64_t wend, const uint8_t* raw, int64_t at,
                                int64_t n) {
  uint32_t c = 0;
  int64_t i = 0;
  for (; i + 8 <= n; i += 8) {
    const int64_t b = at + i / 8;
    c += __popc(b >= wbase && b < wend ? win_byte(win, b - wbase) : raw[b]);
  }
  if (i < n) {
    const int64_t b = at + i / 8;
    const uint32_t x = b >= wbase && b < wend ? win_byte(win, b - wbase) : raw[b];
    c += __popc(x & ((1u << (n - i)) - 1u));
  }
  return c;
}

// One 64-lane workgroup per (data page, stream): stream 0 the definition
// levels, stream 1 the dictionary indices.
__global__ __launch_bounds__(64) void k_pq_walk(const PqPage* pages, const PqSpan* spans, int npages,
                                                const uint8_t* raw, PqRun* runs, int32_t* nruns, PqCk* cks,
                                                PqHeader* hdr) {
  __shared__ uint32_t win[kWalkWin / 4 + 4];
  __shared__ int64_t s_pos, s_items, s_before;
  __shared__ int32_t s_nr, s_ck, s_done;
  const int pi = blockIdx.x >> 1, s = blockIdx.x & 1;
  const PqPage pg = pages[pi];
  const PqSpan sp = spans[pi];
  if (pg.kind != kPqDataPage) return;
  if (s == 0 && sp.def_off < 0) return;
  if (s == 1 && pg.encoding != kPqRleDictionary) return;
  const int64_t end = s == 0 ? sp.def_end : sp.val_end;
  int bw = 1;
  if (s == 1) {
    if (sp.val_off >= sp.val_end) return;  // no values: the run count stays 0
    bw = raw[sp.val_off];  // the index bit width leads the stream
    if (bw > 32) {
      if (threadIdx.x == 0) pq_error(hdr, TQ_EINVAL);
      return;
    }
  }
  const int64_t limit = pg.nrows;  // items: the page's rows (levels), at most that many values
  PqRun* R = runs + (s ? pg.runs_val : pg.runs_def);
  PqCk* C = cks + (s ? pg.ck_val : pg.ck_def);
  const int64_t nck = ((int64_t)pg.nrows + kPqTile - 1) / kPqTile;
  const int vbytes = (bw + 7) / 8;
  if (threadIdx.x == 0) {
    s_pos = s == 0 ? sp.def_off : sp.val_off + 1;
    s_items = 0;
    s_before = 0;
    s_nr = 0;
    s_ck = 0;
    s_done = 0;
  }
  __syncthreads();
  while (!s_done) {
    const int64_t wbase = s_pos & ~(int64_t)3;
    const int64_t wend = wbase + kWalkWin;
    for (int i = threadIdx.x; i < kWalkWin / 4 + 4; i += 64) {
      const int64_t a = wbase + 4 * (int64_t)i;
      win[i] = a < end ? *reinterpret_cast<const uint32_t*>(raw + a) : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t pos = s_pos, items = s_items, before = s_before;
      int32_t nr = s_nr, ck = s_ck;
      bool done = false, bad = false;
      // a run is walked here while its header and fixed bytes lie in the window
      while (!done && !bad) {
        if (items >= limit || pos >= end) {
          done = true;
          break;
        }
        if (pos + 16 > wend) break;  // refill the window from this header
        uint64_t h = 0;
        int sh = 0;
        uint32_t b;
        do {
          b = win_byte(win, pos - wbase);
          h |= (uint64_t)(b & 0x7f) << sh;
          sh += 7;
          pos++;
        } while ((b & 0x80) && sh < 35);
        if (b & 0x80) {
          bad = true;
          break;
        }
        PqRun r;
        r.first = (int32_t)items;
        r.before = (int32_t)before;
        int64_t count, ones;
        if (h & 1) {  // bit-packed: (h >> 1) groups of 8 items, bw bytes each
          const int64_t groups = (int64_t)(h >> 1);
          count = groups * 8;
          r.meta = 0x80000000u | (uint32_t)bw;
          r.arg = pos;
          const int64_t bytes = groups * bw;
          if (groups == 0 || pos + bytes > end) {
            bad = true;
            break;
          }
          const int64_t live = min(count, limit - items);  // the last run is padded to whole groups
          ones = s == 0 ? ones_prefix(win, wbase, wend, raw, pos, live) : 0;
          // checkpoints inside the run
          while (ck < nck && (int64_t)ck * kPqTile < items + count) {
            const int64_t k = (int64_t)ck * kPqTile - items;
            C[ck] = PqCk{nr, (int32_t)(before + (s == 0 ? ones_prefix(win, wbase, wend, raw, pos, k) : 0))};
            ck++;
          }
          pos += bytes;
        } else {  // RLE: (h >> 1) copies of one value of vbytes bytes
          count = (int64_t)(h >> 1);
          if (count == 0 || pos + vbytes > end) {
            bad = true;
            break;
          }
          uint64_t v = 0;
          for (int i = 0; i < vbytes; i++) v |= (uint64_t)win_byte(win, pos - wbase + i) << (8 * i);
          r.meta = (uint32_t)bw;
          r.arg = (int64_t)v;
          ones = s == 0 && v ? min(count, limit - items) : 0;
          while (ck < nck && (int64_t)ck * kPqTile < items + count) {
            const int64_t k = (int64_t)ck * kPqTile - items;
            C[ck] = PqCk{nr, (int32_t)(before + (s == 0 && v ? k : 0))};
            ck++;
          }
          pos += vbytes;
        }
        if (nr >= (s ? pg.max_val : pg.max_def) || items + count > (int64_t)INT32_MAX) {
          bad = true;
          break;
        }
        r.count = (int32_t)count;
        R[nr++] = r;
        items += count;
        before += ones;
      }
      if (bad) pq_error(hdr, TQ_EINVAL);
      if (done || bad) {
        nruns[2 * pi + s] = bad ? 0 : nr;
        if (s == 0 && !bad && items < limit) pq_error(hdr, TQ_EINVAL);  // levels end early
      }
      s_pos = pos;
      s_items = items;
      s_before = before;
      s_nr = nr;
      s_ck = ck;
      s_done = done || bad;
    }
    __syncthreads();
  }
}

// The value of item i of a run (bit width <= 32).
__device__ __forceinline__ uint32_t run_item(const PqRun& r, const uint8_t* raw, int64_t i) {
  if (!(r.meta >> 31)) return (uint32_t)r.arg;
  const uint32_t bw = r.meta & 0xffu;
  const int64_t bit = i * bw;
  const uint64_t x = ld_le(raw, r.arg + (bit >> 3), 8);
  const uint64_t v = x >> (bit & 7);
  return bw == 32 ? (uint32_t)v : (uint32_t)(v & ((1ull << bw) - 1ull));
}

// Index of the run (among n staged in LDS) holding item `item`.
__device__ __forceinline__ int find_run(const PqRun* r, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].first <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Stages in LDS the runs of a table (`total` runs) that hold items
// [first_item, last_item], searching for the first of them from run
// `from` on (a checkpoint's run, at or before it); returns how many, 0 if the
// table does not hold those items.
__device__ int stage_runs(PqRun* dst, const PqRun* src, int32_t from, int32_t total, int64_t first_item,
                          int64_t last_item, int* s_at, int* s_n) {
  if (from < 0 || from > total) from = 0;  // a checkpoint the walk never wrote (it stopped on an error)
  if (threadIdx.x == 0) *s_at = -1;
  __syncthreads();
  int32_t at = -1;
  for (int32_t base = from; base < total; base += kDecBlock) {
    const int32_t i = base + (int32_t)threadIdx.x;
    if (i < total && src[i].first <= first_item && first_item < (int64_t)src[i].first + src[i].count) *s_at = i;
    __syncthreads();
    at = *s_at;
    __syncthreads();  // read by all before anyone writes it again
    if (at >= 0) break;
  }
  if (at < 0) return 0;
  int n = 0;
  for (;;) {
    const int take = min(kDecBlock, min(kTileRuns - n, total - at - n));
    if (take <= 0) break;
    if ((int)threadIdx.x < take) dst[n + threadIdx.x] = src[at + n + threadIdx.x];
    __syncthreads();
    n += take;
    const PqRun& tail = dst[n - 1];
    if ((int64_t)tail.first + tail.count > last_item) break;
  }
  if (threadIdx.x == 0) *s_n = n;
  __syncthreads();
  const int got = *s_n;
  __syncthreads();  // every thread has read *s_at and *s_n before they are reused
  return (int64_t)dst[got - 1].first + dst[got - 1].count > last_item ? got : 0;
}

struct PqOut {
  void* data[TQ_MAX_COLS];
  uint32_t* valid[TQ_MAX_COLS];
};

__global__ __launch_bounds__(kDecBlock) void k_pq_decode(const PqPage* pages, const PqSpan* spans,
                                                         const int32_t* tile_page,
                                                         const uint8_t* raw, const uint8_t* dict, const PqRun* runs,
                                                         const int32_t* nruns, const PqCk* cks, PqOut out,
                                                         PqHeader* hdr) {
  __shared__ PqRun lr[kTileRuns];
  __shared__ int64_t ws[kDecBlock / kWave];
  __shared__ uint32_t bits[kPqTile / 32];
  __shared__ int s_n, s_at;
  const int pi = tile_page[blockIdx.x];
  const PqPage pg = pages[pi];
  const PqSpan sp = spans[pi];
  const int64_t k = blockIdx.x - pg.tile0;
  const int64_t t0 = k * kPqTile;  // first row of the tile in the page
  const int tid = threadIdx.x;
  const int rows = (int)min((int64_t)kPqTile, (int64_t)pg.nrows - t0);
  const bool optional = sp.def_off >= 0;
  // levels: present bits of this thread's rows
  uint32_t present = 0;  // bit i: row tid * kDecRows + i
  int64_t pres0 = t0;    // present rows of the page before the tile
  if (optional) {
    const PqCk c = cks[pg.ck_def + k];
    pres0 = c.before;
    const int n = stage_runs(lr, runs + pg.runs_def, c.run, nruns[2 * pi], t0, t0 + rows - 1, &s_at, &s_n);
    if (n == 0) {
      if (tid == 0) pq_error(hdr, TQ_EINVAL);
      return;
    }
#pragma unroll
    for (int i = 0; i < kDecRows; i++) {
      const int j = tid * kDecRows + i;
      if (j < rows) {
        const int64_t item = t0 + j;
        const PqRun& r = lr[find_run(lr, n, item)];
        if (item < r.first || item >= (int64_t)r.first + r.count) pq_error(hdr, TQ_EINVAL);
        else present |= (run_item(r, raw, item - r.first) & 1u) << i;
      }
    }
    __syncthreads();  // the level runs are read; the table is staged anew below
  } else {
#pragma unroll
    for (int i = 0; i < kDecRows; i++) present |= (uint32_t)(tid * kDecRows + i < rows) << i;
  }
  int64_t excl;
  const int64_t tile_present = block_excl_scan((int64_t)__popc(present), &excl, ws);
  const int64_t v0 = pres0 + excl;  // value index of this thread's first present row
  // values
  uint64_t val[kDecRows];
#pragma unroll
  for (int i = 0; i < kDecRows; i++) val[i] = 0;
  const int w = pg.width;
  if (pg.encoding == kPqPlain) {
    int64_t v = v0;
#pragma unroll
    for (int i = 0; i < kDecRows; i++) {
      if (present >> i & 1u) {
        const int64_t at = sp.val_off + v * w;
        if (at + w > sp.val_end) pq_error(hdr, TQ_EINVAL);
        else val[i] = ld_le(raw, at, w);
        v++;
      }
    }
  } else if (tile_present > 0) {
    const int64_t vfirst = pres0, vlast = pres0 + tile_present - 1;
    const int32_t nv = nruns[2 * pi + 1];
    const PqCk c = cks[pg.ck_val + vfirst / kPqTile];
    // from the checkpoint's run to the one holding vfirst, then the tile's runs
    const int n = stage_runs(lr, runs + pg.runs_val, c.run, nv, vfirst, vlast, &s_at, &s_n);
    if (n == 0) {
      if (tid == 0) pq_error(hdr, TQ_EINVAL);
      return;
    }
    const int64_t* d64 = reinterpret_cast<const int64_t*>(dict + pg.dict_off);
    const int32_t* d32 = reinterpret_cast<const int32_t*>(dict + pg.dict_off);
    int64_t v = v0;
#pragma unroll
    for (int i = 0; i < kDecRows; i++) {
      if (present >> i & 1u) {
        const PqRun& r = lr[find_run(lr, n, v)];
        const bool in_run = v >= r.first && v < (int64_t)r.first + r.count;
        const uint32_t idx = in_run ? run_item(r, raw, v - r.first) : 0u;
        if (!in_run || idx >= (uint32_t)pg.dict_n) pq_error(hdr, TQ_EINVAL);
        else val[i] = w == 8 ? (uint64_t)d64[idx] : (uint64_t)(uint32_t)d32[idx];
        v++;
      }
    }
  }
  // write the values (NULL rows: 0)
  const int64_t row = pg.row0 + t0 + (int64_t)tid * kDecRows;
#pragma unroll
  for (int i = 0; i < kDecRows; i++) {
    if (tid * kDecRows + i < rows) {
      if (w == 8) static_cast<uint64_t*>(out.data[pg.col])[row + i] = val[i];
      else static_cast<uint32_t*>(out.data[pg.col])[row + i] = (uint32_t)val[i];
    }
  }
  // validity: the tile's bits gathered in LDS, then OR-ed into the output words
  uint32_t* vout = out.valid[pg.col];
  if (vout) {
    if (tid < kPqTile / 32) bits[tid] = 0u;
    __syncthreads();
    if (present) atomicOr(&bits[(tid * kDecRows) / 32], present << ((tid * kDecRows) % 32));
    __syncthreads();
    const int64_t base = pg.row0 + t0;      // output bit of tile row 0
    const int64_t w0 = base >> 5, sh = base & 31;
    const int nw = (int)(((base + rows - 1) >> 5) - w0 + 1);
    if (tid < nw) {
      // output word w0 + tid holds tile bits [32 * tid - sh, 32 * tid - sh + 32)
      const int64_t lo_bit = 32 * (int64_t)tid - sh;
      uint32_t x = 0;
      const int64_t i0 = lo_bit >> 5;  // may be -1
      const uint32_t s2 = (uint32_t)(lo_bit & 31);
      const uint32_t a = i0 >= 0 && i0 < kPqTile / 32 ? bits[i0] : 0u;
      const uint32_t b = i0 + 1 >= 0 && i0 + 1 < kPqTile / 32 ? bits[i0 + 1] : 0u;
      x = s2 ? (a >> s2) | (b << (32 - s2)) : a;
      if (x) atomicOr(&vout[w0 + tid], x);
    }
  }
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_parquet_decode(tq_preload* p, void* d_work, size_t work_bytes, const tq_col* out, hipStream_t stream) {
  if (!p || !d_work || !out) return fail(TQ_EINVAL, "preload, work buffer or outputs NULL");
  if ((uintptr_t)d_work & 255) return fail(TQ_EINVAL, "work buffer not 256-byte aligned");
  tq_status s;
  if ((s = pq_join(p))) return s;
  if ((s = pq_parse_pages(p))) return s;
  if (p->decoded) return fail(TQ_EINVAL, "the preload was decoded already");
  const PqLayout L = pq_layout(p);
  if (work_bytes < L.total) return fail(TQ_EINVAL, "work buffer needs %zu bytes", L.total);
  const int32_t ncol = (int32_t)p->cols.size();
  PqOut po{};
  for (int32_t c = 0; c < ncol; c++) {
    const char* name;
    int32_t type, nullable;
    tq_parquet_column(p->pq, p->cols[(size_t)c], &name, &type, &nullable);
    if (out[c].type != type) return fail(TQ_EINVAL, "output %d (%s): type %d, the column is %d", c, name, out[c].type, type);
    if (p->rows > 0 && !out[c].data) return fail(TQ_EINVAL, "output %d (%s): NULL data", c, name);
    if ((uintptr_t)out[c].data & (uintptr_t)(type - 1)) return fail(TQ_EINVAL, "output %d: data not aligned to its width", c);
    if (nullable && !out[c].valid && p->rows > 0)
      return fail(TQ_EINVAL, "output %d (%s) may hold NULLs: it needs a validity bitmap", c, name);
    if ((uintptr_t)out[c].valid & 3) return fail(TQ_EINVAL, "output %d: bitmap not 4-byte aligned", c);
    po.data[c] = const_cast<void*>(out[c].data);
    po.valid[c] = reinterpret_cast<uint32_t*>(const_cast<uint8_t*>(out[c].valid));
  }
  char* W = static_cast<char*>(d_work);
  uint8_t* raw = reinterpret_cast<uint8_t*>(W + L.raw);
  PqHeader* hdr = reinterpret_cast<PqHeader*>(W);
  // host tables: descriptors with offsets made absolute where the kernels want
  // them, the tile -> page map, the dictionary pages; staged through pool pages
  std::vector<PqPage> pages = p->pages;
  std::vector<int32_t> tile_page((size_t)p->tiles), dict_pages, comp_pages, frag_cpage((size_t)p->frags);
  for (size_t i = 0; i < pages.size(); i++) {
    const PqPage& d = pages[i];
    if (d.c_len > 0) {
      for (int64_t f = 0; f < (d.u_len + 65535) / 65536; f++) frag_cpage[(size_t)(d.frag0 + f)] = (int32_t)comp_pages.size();
      comp_pages.push_back((int32_t)i);
    }
    if (d.kind == kPqDictionaryPage) dict_pages.push_back((int32_t)i);
    else
      for (int64_t t = 0; t < ((int64_t)d.nrows + kPqTile - 1) / kPqTile; t++) tile_page[(size_t)(d.tile0 + t)] = (int32_t)i;
  }
  const size_t pb = tq_pagepool_page_bytes(p->pool);
  const size_t host_bytes = pages.size() * sizeof(PqPage) + tile_page.size() * 4 + dict_pages.size() * 4 +
                            comp_pages.size() * 4 + frag_cpage.size() * 4 + 64;
  const int64_t hpages = (int64_t)((host_bytes + pb - 1) / pb);
  std::vector<int32_t> staging((size_t)hpages);
  if (hpages > 0 && tq_pagepool_alloc(p->pool, hpages, staging.data()) != TQ_OK)
    return fail(TQ_ENOMEM, "no free pool page to stage %zu bytes of page tables", host_bytes);
  const size_t tiles_at = L.tiles, dictl_at = L.dictl;
  auto give_back = [&] {
    if (hpages > 0) tq_pagepool_free(p->pool, staging.data(), hpages);
  };
  // copies: the raw bytes page by page, then the tables
  hipError_t e = hipSuccess;
  for (const tq_parquet_read& r : p->reads) {
    int64_t done = 0;
    for (int32_t id : r.pages) {
      const int64_t n = std::min<int64_t>((int64_t)pb, r.bytes - done);
      if (e == hipSuccess)
        e = hipMemcpyAsync(raw + r.raw_off + done, tq_pagepool_page(p->pool, id), (size_t)n, hipMemcpyHostToDevice, stream);
      done += n;
    }
  }
  {
    // pack the three tables into the staging pages back to back, then copy each table
    std::vector<char> blob(host_bytes, 0);
    size_t o = 0;
    const size_t o_pages = o;
    memcpy(blob.data() + o, pages.data(), pages.size() * sizeof(PqPage));
    o += pages.size() * sizeof(PqPage);
    const size_t o_tiles = o;
    memcpy(blob.data() + o, tile_page.data(), tile_page.size() * 4);
    o += tile_page.size() * 4;
    const size_t o_dict = o;
    memcpy(blob.data() + o, dict_pages.data(), dict_pages.size() * 4);
    o += dict_pages.size() * 4;
    const size_t o_comp = o;
    memcpy(blob.data() + o, comp_pages.data(), comp_pages.size() * 4);
    o += comp_pages.size() * 4;
    const size_t o_fcp = o;
    memcpy(blob.data() + o, frag_cpage.data(), frag_cpage.size() * 4);
    o += frag_cpage.size() * 4;
    for (int64_t i = 0; i < hpages; i++) {
      const size_t at = (size_t)i * pb, n = std::min(pb, o > at ? o - at : 0);
      if (n) memcpy(tq_pagepool_page(p->pool, staging[(size_t)i]), blob.data() + at, n);
    }
    // a host range [a, a + n) of the blob to device offset d
    auto copy = [&](size_t a, size_t n, size_t d) {
      while (n > 0 && e == hipSuccess) {
        const size_t pg = a / pb, in = a % pb, take = std::min(n, pb - in);
        e = hipMemcpyAsync(W + d, static_cast<char*>(tq_pagepool_page(p->pool, staging[pg])) + in, take,
                           hipMemcpyHostToDevice, stream);
        a += take;
        d += take;
        n -= take;
      }
    };
    copy(o_pages, pages.size() * sizeof(PqPage), L.pages);
    copy(o_tiles, tile_page.size() * 4, tiles_at);
    copy(o_dict, dict_pages.size() * 4, dictl_at);
    copy(o_comp, comp_pages.size() * 4, L.compl_);
    copy(o_fcp, frag_cpage.size() * 4, L.frag_cp);
  }
  hipEvent_t copied = nullptr;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&copied, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(copied, stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_pq_init, dim3(1), dim3(1), 0, stream, hdr);
    for (int32_t c = 0; c < ncol; c++)
      if (po.valid[c]) {
        const int64_t words = (p->rows + 31) / 32;
        hipLaunchKernelGGL(k_pq_zero, dim3((int)std::max<int64_t>(1, std::min<int64_t>((words + 255) / 256, 1024))),
                           dim3(256), 0, stream, po.valid[c], words);
      }
    // run counts and checkpoints start at zero: a walk that stops on an error leaves them so
    const int64_t zwords = (int64_t)(L.runs - L.nruns) / 4;
    hipLaunchKernelGGL(k_pq_zero, dim3((int)std::max<int64_t>(1, std::min<int64_t>((zwords + 255) / 256, 1024))),
                       dim3(256), 0, stream, reinterpret_cast<uint32_t*>(W + L.nruns), zwords);
    const PqPage* dp = reinterpret_cast<const PqPage*>(W + L.pages);
    PqSpan* spans = reinterpret_cast<PqSpan*>(W + L.spans);
    if (!comp_pages.empty()) {
      const int32_t* cl = reinterpret_cast<const int32_t*>(W + L.compl_);
      int32_t* frag_in = reinterpret_cast<int32_t*>(W + L.frag_in);
      int32_t* flags = reinterpret_cast<int32_t*>(W + L.cflags);
      hipLaunchKernelGGL(k_pq_snappy_scan, dim3((int)comp_pages.size()), dim3(64 * kScanWaves), 0, stream, dp, cl, raw, frag_in,
                         flags, hdr);
      if (p->frags > 0)
        hipLaunchKernelGGL(k_pq_snappy_frag, dim3((int)p->frags), dim3(2 * kWave), 0, stream, dp, cl,
                           reinterpret_cast<const int32_t*>(W + L.frag_cp), raw, frag_in, flags, hdr);
      hipLaunchKernelGGL(k_pq_snappy, dim3((int)comp_pages.size()), dim3(64), 0, stream, dp, cl, raw, flags, hdr);
    }
    if (!pages.empty())
      hipLaunchKernelGGL(k_pq_span, dim3((int)std::min<size_t>((pages.size() + 255) / 256, 1024)), dim3(256), 0,
                         stream, dp, (int)pages.size(), raw, spans, hdr);
    if (!dict_pages.empty())
      hipLaunchKernelGGL(k_pq_dict, dim3((int)dict_pages.size() * kDictBlocks), dim3(kDecBlock), 0, stream, dp,
                         reinterpret_cast<const int32_t*>(W + dictl_at), raw, reinterpret_cast<uint8_t*>(W + L.dict));
    if (!pages.empty())
      hipLaunchKernelGGL(k_pq_walk, dim3((int)(2 * pages.size())), dim3(64), 0, stream, dp, spans, (int)pages.size(), raw,
                         reinterpret_cast<PqRun*>(W + L.runs), reinterpret_cast<int32_t*>(W + L.nruns),
                         reinterpret_cast<PqCk*>(W + L.cks), hdr);
    if (p->tiles > 0)
      hipLaunchKernelGGL(k_pq_decode, dim3((int)p->tiles), dim3(kDecBlock), 0, stream, dp, spans,
                         reinterpret_cast<const int32_t*>(W + tiles_at), raw, reinterpret_cast<const uint8_t*>(W + L.dict),
                         reinterpret_cast<const PqRun*>(W + L.runs), reinterpret_cast<const int32_t*>(W + L.nruns),
                         reinterpret_cast<const PqCk*>(W + L.cks), po, hdr);
    e = hipGetLastError();
  }
  // the pool pages may be reused once the copies out of them have finished
  hipError_t e2 = copied ? hipEventSynchronize(copied) : hipSuccess;
  if (copied) (void)hipEventDestroy(copied);
  if (e2 != hipSuccess && copied) {
    // the copies' fate is unknown: keep the pages rather than hand them out again
    return hip_fail(e2, "waiting for the page copies");
  }
  give_back();
  pq_release_pages(p);
  p->decoded = true;
  if (e != hipSuccess) return hip_fail(e, "parquet decode");
  return TQ_OK;
}

}  // extern "C"
