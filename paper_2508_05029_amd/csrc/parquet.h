// Parquet scan: the host side (file metadata, byte ranges, page headers) and
// the page descriptors the decode kernels read.
#pragma once

#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tq.h"

namespace tq {

// Enumerations of the Parquet format (its Thrift definitions).
enum PqType : int32_t { kPqBoolean = 0, kPqInt32 = 1, kPqInt64 = 2 };
enum PqRepetition : int32_t { kPqRequired = 0, kPqOptional = 1, kPqRepeated = 2 };
enum PqEncoding : int32_t { kPqPlain = 0, kPqPlainDictionary = 2, kPqRle = 3, kPqRleDictionary = 8 };
enum PqPageType : int32_t { kPqDataPage = 0, kPqIndexPage = 1, kPqDictionaryPage = 2, kPqDataPageV2 = 3 };
enum PqCodec : int32_t { kPqUncompressed = 0, kPqSnappy = 1 };
constexpr int64_t kPqLevelsInBody = -2;  // def_off of a v1 page: the levels lead its body, after a 4-byte length

struct PqColumn {
  std::string name;
  int32_t type = -1;
  int32_t repetition = kPqRequired;
};

struct PqChunk {
  int64_t start = 0;  // first byte of the chunk (its dictionary page, else its first data page)
  int64_t bytes = 0;  // total_compressed_size
  int32_t codec = 0;
  int64_t num_values = 0;
};

struct PqRowGroup {
  int64_t num_rows = 0;
  std::vector<PqChunk> chunks;  // one per column
};

// One page as the kernels see it. Offsets are bytes from the start of the
// raw area of the device work buffer (the decompressed area follows it).
struct PqPage {
  int64_t row0;        // first output row (rows of all selected row groups, in order)
  int32_t nrows;       // rows (= level count of a flat column)
  int32_t col;         // output column (index into the call's column list)
  int64_t def_off;     // definition levels (RLE/bit-packed hybrid, bit width 1); -1: none (a required
  int64_t def_end;     // column); kPqLevelsInBody: they lead the body [val_off, val_end)
  int64_t val_off;     // values section (or the whole body, see def_off)
  int64_t val_end;
  int64_t c_off, c_len;  // a Snappy-compressed body: its bytes in the raw area (c_len 0: not compressed)
  int64_t u_off, u_len;  // and where it is inflated to (= val_off)
  int64_t frag0;         // its first 64 KiB output fragment (compressed bodies)
  int32_t encoding;    // kPqPlain, or dictionary indices (kPqRleDictionary)
  int32_t width;       // 4 or 8 bytes
  int64_t dict_off;    // dictionary values (aligned copy), from the dictionary area's start; -1 if none
  int32_t dict_n;      // entries
  int32_t kind;        // kPqDataPage, kPqDictionaryPage
  int64_t runs_def;    // offsets (in PqRun units) of this page's run tables
  int64_t runs_val;
  int64_t max_def;     // their capacities
  int64_t max_val;
  int64_t ck_def;      // offsets (in PqCk units) of its checkpoints, one per kPqTile items
  int64_t ck_val;
  int64_t tile0;       // its first decode tile (data pages)
};

constexpr int kPqTile = 1024;  // rows per decode workgroup, and the checkpoint spacing

// A data page's level and value sections, fixed on the device once the page
// is inflated (a v1 page's level length is inside its body).
struct PqSpan {
  int64_t def_off, def_end, val_off, val_end;
};

// Where item k * kPqTile of a stream lies: run `run`, with `before` items
// equal to 1 ahead of it (definition levels: present rows before that row).
struct PqCk {
  int32_t run, before;
};

// A run of an RLE/bit-packed hybrid stream: items [first, first + count);
// bit-packed (meta >> 31) at byte `arg` of the raw area, else the repeated
// value `arg`; meta & 0xff is the bit width; `before`: items equal to 1 in
// the runs ahead of this one (definition levels: present rows before it).
struct PqRun {
  int32_t first, count;
  uint32_t meta;
  int32_t before;
  int64_t arg;
};

}  // namespace tq

struct tq_parquet {
  int fd = -1;
  std::string path;
  int64_t file_size = 0;
  int64_t num_rows = 0;
  std::vector<tq::PqColumn> cols;
  std::vector<tq::PqRowGroup> rgs;
};

struct tq_parquet_read {
  int64_t file_off, bytes;   // the merged byte range
  int64_t raw_off;           // where it lands in the raw area
  std::vector<int32_t> pages;  // pool pages holding it, in order
};

// A piece of a read: at most kPqReadPiece bytes inside one pool page.
struct tq_parquet_piece {
  int64_t file_off, bytes;
  char* dst;
};

struct tq_preload {
  tq_parquet* pq = nullptr;
  tq_pagepool* pool = nullptr;
  int32_t rg0 = 0, rg1 = 0;
  std::vector<int32_t> cols;
  std::vector<tq_parquet_read> reads;
  int64_t raw_bytes = 0;
  int64_t rows = 0;
  std::vector<tq_parquet_piece> pieces;
  std::vector<std::thread> readers;  // each takes the next piece until none is left
  std::atomic<int64_t> next_piece{0};
  std::atomic<bool> read_failed{false};
  std::mutex read_mu;  // guards read_status / read_error
  bool joined = false;
  bool decoded = false;  // a preload is decoded once: its pages go back to the pool
  tq_status read_status = TQ_OK;
  std::string read_error;
  // page headers, parsed once the bytes are in host memory
  bool parsed = false;
  std::vector<tq::PqPage> pages;
  int64_t decomp_bytes = 0;
  int64_t dict_bytes = 0;
  int64_t run_slots = 0;
  int64_t ck_slots = 0;
  int64_t tiles = 0;
  int64_t frags = 0;  // 64 KiB output fragments of the compressed bodies
};

namespace tq {
tq_status pq_parse_pages(tq_preload* p);
size_t pq_work_bytes(const tq_preload* p);
tq_status pq_join(tq_preload* p);
void pq_release_pages(tq_preload* p);

// Device work buffer of a decode: header | raw bytes | inflated page bodies |
// dictionaries | page descriptors | spans | run counts | checkpoints | run
// tables | tile -> page map | dictionary page list | compressed page list |
// their scan flags | fragment starts | fragment -> compressed page map (each
// part 256-aligned).
struct PqLayout {
  size_t raw, dict, pages, spans, nruns, cks, runs, tiles, dictl, compl_, cflags, frag_in, frag_cp, total;
};
PqLayout pq_layout(const tq_preload* p);
}  // namespace tq
