// Parquet scan, host side: the file footer (Thrift compact protocol), the
// byte ranges of the column chunks a scan needs, merged when close (Byte
// Range Pre-loading, Section 3.3.3), read ahead into pool pages by threads
// of their own, and the page headers walked once the bytes are in host
// memory. The pages themselves are decoded on the GPU (parquet.hip).
#include "parquet.h"

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <system_error>

#include "common.h"

namespace tq {

// ------------------------------------------------------- Thrift compact protocol

namespace {

enum TType : int { kStop = 0, kTrue = 1, kFalse = 2, kByte = 3, kI16 = 4, kI32 = 5, kI64 = 6, kDouble = 7,
                   kBinary = 8, kList = 9, kSet = 10, kMap = 11, kStruct = 12 };

// Reads one Thrift struct after another from a byte buffer; any malformed or
// truncated input sets `bad` and yields zeros from then on.
struct Thrift {
  const uint8_t* p;
  const uint8_t* end;
  bool bad = false;

  uint8_t byte() {
    if (p >= end) {
      bad = true;
      return 0;
    }
    return *p++;
  }
  uint64_t varint() {
    uint64_t v = 0;
    for (int shift = 0; shift < 64; shift += 7) {
      const uint8_t b = byte();
      v |= (uint64_t)(b & 0x7f) << shift;
      if (!(b & 0x80)) return v;
    }
    bad = true;
    return 0;
  }
  int64_t zigzag() {
    const uint64_t u = varint();
    return (int64_t)(u >> 1) ^ -(int64_t)(u & 1);
  }
  std::string binary() {
    const uint64_t n = varint();
    if (n > (uint64_t)(end - p)) {
      bad = true;
      return std::string();
    }
    std::string s(reinterpret_cast<const char*>(p), (size_t)n);
    p += n;
    return s;
  }
  // A field header: false at the struct's end (kStop).
  bool field(int16_t& id, int& type) {
    const uint8_t b = byte();
    if (bad || b == 0) return false;
    type = b & 0x0f;
    const int delta = b >> 4;
    id = delta ? (int16_t)(id + delta) : (int16_t)zigzag();
    return true;
  }
  // List or set header: element type and count.
  void list(int& etype, int64_t& n) {
    const uint8_t b = byte();
    etype = b & 0x0f;
    n = (b >> 4) == 0x0f ? (int64_t)varint() : (int64_t)(b >> 4);
    if (n < 0 || n > (int64_t)(end - p)) {  // every element takes at least a byte
      bad = true;
      n = 0;
    }
  }
  void skip(int type, int depth = 0) {
    if (bad || depth > 32) {
      bad = true;
      return;
    }
    switch (type) {
      case kTrue:
      case kFalse:
        break;  // a struct field's value is in its type
      case kByte:
        byte();
        break;
      case kI16:
      case kI32:
      case kI64:
        varint();
        break;
      case kDouble:
        for (int i = 0; i < 8; i++) byte();
        break;
      case kBinary: {
        const uint64_t n = varint();
        if (n > (uint64_t)(end - p)) bad = true;
        else p += n;
        break;
      }
      case kList:
      case kSet: {
        int et;
        int64_t n;
        list(et, n);
        for (int64_t i = 0; i < n && !bad; i++) {
          if (et == kTrue || et == kFalse) byte();  // a bool element is one byte
          else skip(et, depth + 1);
        }
        break;
      }
      case kMap: {
        const int64_t n = (int64_t)varint();
        if (n > 0) {
          const uint8_t kv = byte();
          for (int64_t i = 0; i < n && !bad; i++) {
            skip(kv >> 4, depth + 1);
            skip(kv & 0x0f, depth + 1);
          }
        }
        break;
      }
      case kStruct: {
        int16_t id = 0;
        int t;
        while (field(id, t)) skip(t, depth + 1);
        break;
      }
      default:
        bad = true;
    }
  }
  int64_t integer(int type) { return (type == kI16 || type == kI32 || type == kI64) ? zigzag() : (skip(type), 0); }
};

struct ColumnMeta {
  int32_t type = -1, codec = 0;
  int64_t num_values = 0, total_compressed = 0, data_page_offset = -1, dictionary_page_offset = -1;
};

void read_column_meta(Thrift& t, ColumnMeta& m) {
  int16_t id = 0;
  int type;
  while (t.field(id, type)) {
    switch (id) {
      case 1: m.type = (int32_t)t.integer(type); break;
      case 4: m.codec = (int32_t)t.integer(type); break;
      case 5: m.num_values = t.integer(type); break;
      case 7: m.total_compressed = t.integer(type); break;
      case 9: m.data_page_offset = t.integer(type); break;
      case 11: m.dictionary_page_offset = t.integer(type); break;
      default: t.skip(type);
    }
  }
}

bool read_chunk(Thrift& t, PqChunk& c) {
  int16_t id = 0;
  int type;
  ColumnMeta m;
  bool external = false, have_meta = false;
  while (t.field(id, type)) {
    if (id == 1 && type == kBinary) {
      external = !t.binary().empty();  // the chunk lives in another file
    } else if (id == 3 && type == kStruct) {
      read_column_meta(t, m);
      have_meta = true;
    } else {
      t.skip(type);
    }
  }
  if (external || !have_meta || m.data_page_offset < 0) return false;
  c.start = (m.dictionary_page_offset > 0 && m.dictionary_page_offset < m.data_page_offset) ? m.dictionary_page_offset
                                                                                          : m.data_page_offset;
  c.bytes = m.total_compressed;
  c.codec = m.codec;
  c.num_values = m.num_values;
  return true;
}

bool read_row_group(Thrift& t, PqRowGroup& g) {
  int16_t id = 0;
  int type;
  bool ok = true;
  while (t.field(id, type)) {
    if (id == 1 && type == kList) {
      int et;
      int64_t n;
      t.list(et, n);
      for (int64_t i = 0; i < n && !t.bad; i++) {
        PqChunk c;
        ok = read_chunk(t, c) && ok;
        g.chunks.push_back(c);
      }
    } else if (id == 3) {
      g.num_rows = t.integer(type);
    } else {
      t.skip(type);
    }
  }
  return ok;
}

struct SchemaElement {
  int32_t type = -1, repetition = kPqRequired, num_children = 0;
  std::string name;
};

void read_schema_element(Thrift& t, SchemaElement& e) {
  int16_t id = 0;
  int type;
  while (t.field(id, type)) {
    switch (id) {
      case 1: e.type = (int32_t)t.integer(type); break;
      case 3: e.repetition = (int32_t)t.integer(type); break;
      case 4:
        if (type == kBinary) e.name = t.binary();
        else t.skip(type);
        break;
      case 5: e.num_children = (int32_t)t.integer(type); break;
      default: t.skip(type);
    }
  }
}

struct PageHeader {
  int32_t type = -1, uncompressed = -1, compressed = -1;
  int32_t num_values = 0, encoding = -1, def_encoding = -1;
  int32_t v2_num_nulls = 0, v2_num_rows = 0, v2_def_bytes = 0, v2_rep_bytes = 0;
  bool v2_compressed = true;
  int32_t dict_num_values = 0, dict_encoding = -1;
};

void read_page_header(Thrift& t, PageHeader& h) {
  int16_t id = 0;
  int type;
  while (t.field(id, type)) {
    if (id == 1) h.type = (int32_t)t.integer(type);
    else if (id == 2) h.uncompressed = (int32_t)t.integer(type);
    else if (id == 3) h.compressed = (int32_t)t.integer(type);
    else if ((id == 5 || id == 7 || id == 8) && type == kStruct) {
      int16_t sid = 0;
      int st;
      while (t.field(sid, st)) {
        if (id == 5) {  // DataPageHeader
          if (sid == 1) h.num_values = (int32_t)t.integer(st);
          else if (sid == 2) h.encoding = (int32_t)t.integer(st);
          else if (sid == 3) h.def_encoding = (int32_t)t.integer(st);
          else t.skip(st);
        } else if (id == 7) {  // DictionaryPageHeader
          if (sid == 1) h.dict_num_values = (int32_t)t.integer(st);
          else if (sid == 2) h.dict_encoding = (int32_t)t.integer(st);
          else t.skip(st);
        } else {  // DataPageHeaderV2
          if (sid == 1) h.num_values = (int32_t)t.integer(st);
          else if (sid == 2) h.v2_num_nulls = (int32_t)t.integer(st);
          else if (sid == 3) h.v2_num_rows = (int32_t)t.integer(st);
          else if (sid == 4) h.encoding = (int32_t)t.integer(st);
          else if (sid == 5) h.v2_def_bytes = (int32_t)t.integer(st);
          else if (sid == 6) h.v2_rep_bytes = (int32_t)t.integer(st);
          else if (sid == 7) h.v2_compressed = st == kTrue;
          else t.skip(st);
        }
      }
    } else {
      t.skip(type);
    }
  }
}

int32_t width_of_type(int32_t pq_type) { return pq_type == kPqInt32 ? 4 : pq_type == kPqInt64 ? 8 : 0; }

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// The raw-area bytes [off, off + n) of a preload, copied out of its pool pages.
bool copy_out(const tq_preload* p, int64_t off, int64_t n, uint8_t* dst) {
  const size_t pb = tq_pagepool_page_bytes(p->pool);
  for (const tq_parquet_read& r : p->reads) {
    if (off < r.raw_off || off >= r.raw_off + r.bytes) continue;
    if (off + n > r.raw_off + r.bytes) n = r.raw_off + r.bytes - off;
    int64_t in = off - r.raw_off;
    while (n > 0) {
      const size_t pg = (size_t)in / pb, at = (size_t)in % pb;
      const size_t take = std::min<size_t>((size_t)n, pb - at);
      memcpy(dst, static_cast<char*>(tq_pagepool_page(p->pool, r.pages[pg])) + at, take);
      dst += take;
      in += (int64_t)take;
      n -= (int64_t)take;
    }
    return true;
  }
  return false;
}

// Raw-area offset of file byte `file_off` (inside one of the reads).
int64_t raw_of(const tq_preload* p, int64_t file_off) {
  for (const tq_parquet_read& r : p->reads)
    if (file_off >= r.file_off && file_off < r.file_off + r.bytes) return r.raw_off + (file_off - r.file_off);
  return -1;
}

// Reader threads per preload, and the largest piece one of them reads at a
// time: one thread copies from the page cache at well under the host's memory
// bandwidth, so the merged ranges are split and read by several at once.
constexpr int kPqReaders = 4;
constexpr int64_t kPqReadPiece = 2 << 20;

void read_pieces(tq_preload* p) {
  for (;;) {
    const int64_t t = p->next_piece.fetch_add(1);
    if (t >= (int64_t)p->pieces.size() || p->read_failed.load()) return;
    const tq_parquet_piece& pc = p->pieces[(size_t)t];
    int64_t got = 0;
    while (got < pc.bytes) {
      const ssize_t k = pread(p->pq->fd, pc.dst + got, (size_t)(pc.bytes - got), (off_t)(pc.file_off + got));
      if (k <= 0) {
        std::lock_guard<std::mutex> lock(p->read_mu);
        if (!p->read_status) {
          p->read_status = TQ_EINVAL;
          p->read_error = "reading " + p->pq->path + " failed";
        }
        p->read_failed.store(true);
        return;
      }
      got += k;
    }
  }
}

}  // namespace

// Walks the page headers of every chunk of a finished preload and lays out
// the device work buffer: raw bytes | dictionaries (aligned copies) | page
// descriptors | run tables.
tq_status pq_parse_pages(tq_preload* p) {
  if (p->parsed) return TQ_OK;
  const tq_parquet* pq = p->pq;
  std::vector<uint8_t> hdr;
  int64_t row0 = 0, dict_bytes = 0, run_slots = 0, ck_slots = 0, tiles = 0, decomp_bytes = 0, frags = 0;
  const int64_t decomp_base = align256(p->raw_bytes + 16);  // from the raw area's start
  std::vector<PqPage> pages;
  for (int32_t g = p->rg0; g < p->rg1; g++) {
    const PqRowGroup& rg = pq->rgs[(size_t)g];
    for (size_t ci = 0; ci < p->cols.size(); ci++) {
      const int32_t c = p->cols[ci];
      const PqColumn& col = pq->cols[(size_t)c];
      const PqChunk& ch = rg.chunks[(size_t)c];
      const int32_t width = width_of_type(col.type);
      int64_t at = ch.start, rows = 0, dict_off = -1;
      int32_t dict_n = 0;
      const int64_t end = ch.start + ch.bytes;
      while (at < end) {
        const int64_t raw = raw_of(p, at);
        if (raw < 0) return fail(TQ_EINVAL, "column %d: page at %lld outside the preloaded ranges", c, (long long)at);
        const int64_t avail = std::min<int64_t>(end - at, 1 << 16);
        hdr.resize((size_t)avail);
        if (!copy_out(p, raw, avail, hdr.data())) return fail(TQ_EINVAL, "page header outside the reads");
        Thrift t{hdr.data(), hdr.data() + avail};
        PageHeader h;
        read_page_header(t, h);
        const int64_t hbytes = t.p - hdr.data();
        if (t.bad || h.type < 0 || h.compressed < 0 || at + hbytes + h.compressed > end)
          return fail(TQ_EINVAL, "column %d: malformed page header at byte %lld", c, (long long)at);
        const int64_t data = raw + hbytes;  // the page body in the raw area
        // a compressed body is inflated into the decompressed area (at
        // decomp_base + decomp_bytes), which is where the kernels then read it
        auto inflate = [&](PqPage& d, int64_t c_off, int64_t c_len, int64_t u_len) {
          d.c_off = c_off;
          d.c_len = c_len;
          d.u_len = u_len;
          d.u_off = decomp_base + decomp_bytes;
          decomp_bytes += align256(u_len + 16);
          d.frag0 = frags;
          frags += (u_len + 65535) / 65536;
          return d.u_off;
        };
        const bool snappy = ch.codec == kPqSnappy;
        if (h.uncompressed < 0 || (snappy && h.uncompressed > (1 << 30)))
          return fail(TQ_EINVAL, "column %d: page size %d", c, h.uncompressed);
        if (h.type == kPqDictionaryPage) {
          if (h.dict_encoding != kPqPlain && h.dict_encoding != kPqPlainDictionary)
            return fail(TQ_EINVAL, "column %d: dictionary page encoding %d", c, h.dict_encoding);
          const int64_t body_bytes = snappy ? h.uncompressed : h.compressed;
          if ((int64_t)h.dict_num_values * width > body_bytes || h.dict_num_values < 0)
            return fail(TQ_EINVAL, "column %d: dictionary page too short", c);
          PqPage d{};
          d.kind = kPqDictionaryPage;
          d.col = (int32_t)ci;
          d.val_off = snappy ? inflate(d, data, h.compressed, h.uncompressed) : data;
          d.val_end = d.val_off + body_bytes;
          d.width = width;
          d.dict_off = dict_bytes;  // from the dictionary area's start
          d.dict_n = h.dict_num_values;
          d.def_off = -1;
          pages.push_back(d);
          dict_off = dict_bytes;
          dict_n = h.dict_num_values;
          dict_bytes += align256((int64_t)h.dict_num_values * width);
        } else if (h.type == kPqDataPage || h.type == kPqDataPageV2) {
          PqPage d{};
          d.kind = kPqDataPage;
          d.col = (int32_t)ci;
          d.row0 = row0 + rows;
          d.nrows = h.num_values;
          d.width = width;
          d.encoding = h.encoding == kPqPlainDictionary ? kPqRleDictionary : h.encoding;
          if (d.encoding != kPqPlain && d.encoding != kPqRleDictionary)
            return fail(TQ_EINVAL, "column %d: page encoding %d is not supported", c, h.encoding);
          if (d.encoding == kPqRleDictionary && dict_off < 0)
            return fail(TQ_EINVAL, "column %d: dictionary-encoded page without a dictionary", c);
          if (d.nrows < 0) return fail(TQ_EINVAL, "column %d: negative value count", c);
          d.dict_off = d.encoding == kPqRleDictionary ? dict_off : -1;
          d.dict_n = d.encoding == kPqRleDictionary ? dict_n : 0;
          const bool optional = col.repetition == kPqOptional;
          if (h.type == kPqDataPage) {
            // levels and values are one body (compressed together); the
            // levels' 4-byte length prefix is read on the device
            if (optional && h.def_encoding != kPqRle)
              return fail(TQ_EINVAL, "column %d: level encoding %d", c, h.def_encoding);
            const int64_t body_bytes = snappy ? h.uncompressed : h.compressed;
            d.val_off = snappy ? inflate(d, data, h.compressed, h.uncompressed) : data;
            d.val_end = d.val_off + body_bytes;
            d.def_off = optional ? kPqLevelsInBody : -1;
            d.def_end = -1;
          } else {
            if (h.v2_rep_bytes != 0) return fail(TQ_EINVAL, "column %d: repetition levels", c);
            if (h.v2_def_bytes > 0 && !optional) return fail(TQ_EINVAL, "column %d: levels on a required column", c);
            if (h.v2_def_bytes < 0 || h.v2_def_bytes > h.compressed)
              return fail(TQ_EINVAL, "column %d: level bytes %d", c, h.v2_def_bytes);
            d.def_off = optional ? data : -1;  // the levels are never compressed
            d.def_end = optional ? data + h.v2_def_bytes : -1;
            const int64_t vc = h.compressed - h.v2_def_bytes;
            const int64_t vu = h.uncompressed - h.v2_def_bytes;
            const bool inflated = snappy && h.v2_compressed;
            if (inflated && vu < 0) return fail(TQ_EINVAL, "column %d: page sizes", c);
            d.val_off = inflated ? inflate(d, data + h.v2_def_bytes, vc, vu) : data + h.v2_def_bytes;
            d.val_end = d.val_off + (inflated ? vu : vc);
          }
          // a run covers at least one item and takes at least one byte (its
          // header; levels, of bit width 1, also a value byte or a packed group)
          const int64_t level_bytes = d.def_off == kPqLevelsInBody ? d.val_end - d.val_off : d.def_end - d.def_off;
          d.max_def = optional ? std::min<int64_t>(d.nrows, level_bytes / 2) + 1 : 0;
          d.max_val = d.encoding == kPqRleDictionary ? std::min<int64_t>(d.nrows, d.val_end - d.val_off) + 1 : 0;
          d.runs_def = run_slots;
          d.runs_val = run_slots + d.max_def;
          run_slots += d.max_def + d.max_val;
          const int64_t nck = ((int64_t)d.nrows + kPqTile - 1) / kPqTile;
          d.ck_def = ck_slots;
          d.ck_val = ck_slots + nck;
          ck_slots += 2 * nck;
          d.tile0 = tiles;
          tiles += nck;
          pages.push_back(d);
          rows += h.num_values;
        } else if (h.type != kPqIndexPage) {
          return fail(TQ_EINVAL, "column %d: page type %d", c, h.type);
        }
        at += hbytes + h.compressed;
      }
      if (rows != rg.num_rows)
        return fail(TQ_EINVAL, "column %d of row group %d: %lld rows in its pages, %lld in the row group", c, g,
                    (long long)rows, (long long)rg.num_rows);
    }
    row0 += rg.num_rows;
  }
  p->pages = std::move(pages);
  p->decomp_bytes = decomp_bytes;
  p->dict_bytes = dict_bytes;
  p->run_slots = run_slots;
  p->ck_slots = ck_slots;
  p->tiles = tiles;
  p->frags = frags;
  p->parsed = true;
  return TQ_OK;
}

PqLayout pq_layout(const tq_preload* p) {
  PqLayout L;
  size_t at = 256;  // the header: magic, latched error
  L.raw = at;
  at += (size_t)align256(p->raw_bytes + 16);  // loads may read a few bytes past a stream's end
  at += (size_t)p->decomp_bytes;               // inflated page bodies (each padded likewise)
  L.dict = at;
  at += (size_t)p->dict_bytes;
  L.pages = at;
  at += (size_t)align256((int64_t)(p->pages.size() * sizeof(PqPage)));
  L.spans = at;
  at += (size_t)align256((int64_t)(p->pages.size() * sizeof(PqSpan)));
  L.nruns = at;
  at += (size_t)align256((int64_t)p->pages.size() * 2 * 4);
  L.cks = at;
  at += (size_t)align256(p->ck_slots * (int64_t)sizeof(PqCk));
  L.runs = at;
  at += (size_t)align256(p->run_slots * (int64_t)sizeof(PqRun));
  int64_t ndict = 0;
  for (const PqPage& d : p->pages) ndict += d.kind == kPqDictionaryPage;
  L.tiles = at;
  at += (size_t)align256(p->tiles * 4);
  int64_t ncomp = 0;
  for (const PqPage& d : p->pages) ncomp += d.c_len > 0;
  L.dictl = at;
  at += (size_t)align256(ndict * 4);
  L.compl_ = at;
  at += (size_t)align256(ncomp * 4);
  L.cflags = at;
  at += (size_t)align256(ncomp * 4);
  L.frag_in = at;
  at += (size_t)align256(p->frags * 4);
  L.frag_cp = at;
  at += (size_t)align256(p->frags * 4);
  L.total = at;
  return L;
}

size_t pq_work_bytes(const tq_preload* p) { return pq_layout(p).total; }

tq_status pq_join(tq_preload* p) {
  if (!p->joined) {
    for (std::thread& t : p->readers)
      if (t.joinable()) t.join();
    p->joined = true;
  }
  if (p->read_status) return fail(p->read_status, "%s", p->read_error.c_str());
  return TQ_OK;
}

void pq_release_pages(tq_preload* p) {
  for (tq_parquet_read& r : p->reads) {
    if (!r.pages.empty()) tq_pagepool_free(p->pool, r.pages.data(), (int64_t)r.pages.size());
    r.pages.clear();
  }
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_parquet_open(const char* path, tq_parquet** out) {
  if (!path || !out) return fail(TQ_EINVAL, "path or out is NULL");
  *out = nullptr;
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return fail(TQ_EINVAL, "cannot open %s", path);
  struct stat st;
  auto bad = [&](const char* why) {
    close(fd);
    return fail(TQ_EINVAL, "%s: %s", path, why);
  };
  if (fstat(fd, &st) != 0 || st.st_size < 12) return bad("not a Parquet file (too short)");
  const int64_t size = st.st_size;
  uint8_t tail[8], head[4];
  if (pread(fd, tail, 8, size - 8) != 8 || pread(fd, head, 4, 0) != 4) return bad("read failed");
  if (memcmp(tail + 4, "PAR1", 4) != 0 || memcmp(head, "PAR1", 4) != 0) return bad("no PAR1 magic");
  const int64_t flen = (int64_t)tail[0] | (int64_t)tail[1] << 8 | (int64_t)tail[2] << 16 | (int64_t)tail[3] << 24;
  if (flen <= 0 || flen > size - 12) return bad("footer length outside the file");
  std::vector<uint8_t> footer((size_t)flen);
  if (pread(fd, footer.data(), (size_t)flen, size - 8 - flen) != flen) return bad("footer read failed");
  Thrift t{footer.data(), footer.data() + flen};
  std::vector<SchemaElement> schema;
  std::vector<PqRowGroup> rgs;
  int64_t num_rows = -1;
  bool chunks_ok = true;
  int16_t id = 0;
  int type;
  while (t.field(id, type)) {
    if (id == 2 && type == kList) {
      int et;
      int64_t n;
      t.list(et, n);
      for (int64_t i = 0; i < n && !t.bad; i++) {
        SchemaElement e;
        read_schema_element(t, e);
        schema.push_back(e);
      }
    } else if (id == 3) {
      num_rows = t.integer(type);
    } else if (id == 4 && type == kList) {
      int et;
      int64_t n;
      t.list(et, n);
      for (int64_t i = 0; i < n && !t.bad; i++) {
        PqRowGroup g;
        chunks_ok = read_row_group(t, g) && chunks_ok;
        rgs.push_back(std::move(g));
      }
    } else {
      t.skip(type);
    }
  }
  if (t.bad) return bad("malformed footer");
  if (schema.empty() || num_rows < 0) return bad("footer without schema or row count");
  if (schema[0].num_children != (int32_t)schema.size() - 1) return bad("nested schemas are not supported");
  if (!chunks_ok) return bad("a column chunk without metadata, or in another file");
  auto* pq = new tq_parquet();
  pq->fd = fd;
  pq->path = path;
  pq->file_size = size;
  pq->num_rows = num_rows;
  for (size_t i = 1; i < schema.size(); i++) {
    if (schema[i].num_children != 0 || schema[i].repetition == kPqRepeated) {
      delete pq;
      return bad("nested or repeated columns are not supported");
    }
    pq->cols.push_back(PqColumn{schema[i].name, schema[i].type, schema[i].repetition});
  }
  int64_t total = 0;
  for (const PqRowGroup& g : rgs) {
    if (g.chunks.size() != pq->cols.size()) {
      delete pq;
      return bad("a row group's chunk count differs from the schema");
    }
    for (const PqChunk& c : g.chunks)
      if (c.start < 4 || c.bytes < 0 || c.start + c.bytes > size - 8 - flen) {
        delete pq;
        return bad("a column chunk lies outside the file's data");
      }
    total += g.num_rows;
  }
  if (total != num_rows) {
    delete pq;
    return bad("row groups do not add up to the row count");
  }
  pq->rgs = std::move(rgs);
  *out = pq;
  return TQ_OK;
}

void tq_parquet_close(tq_parquet* pq) {
  if (!pq) return;
  if (pq->fd >= 0) close(pq->fd);
  delete pq;
}

int64_t tq_parquet_num_rows(const tq_parquet* pq) { return pq ? pq->num_rows : -1; }
int32_t tq_parquet_num_row_groups(const tq_parquet* pq) { return pq ? (int32_t)pq->rgs.size() : -1; }
int32_t tq_parquet_num_columns(const tq_parquet* pq) { return pq ? (int32_t)pq->cols.size() : -1; }

int64_t tq_parquet_row_group_rows(const tq_parquet* pq, int32_t rg) {
  if (!pq || rg < 0 || rg >= (int32_t)pq->rgs.size()) return -1;
  return pq->rgs[(size_t)rg].num_rows;
}

tq_status tq_parquet_column(const tq_parquet* pq, int32_t c, const char** name, int32_t* type, int32_t* nullable) {
  if (!pq || c < 0 || c >= (int32_t)pq->cols.size()) return fail(TQ_EINVAL, "no column %d", c);
  const PqColumn& col = pq->cols[(size_t)c];
  if (name) *name = col.name.c_str();
  if (type) *type = width_of_type(col.type);
  if (nullable) *nullable = col.repetition == kPqOptional;
  return TQ_OK;
}

tq_status tq_parquet_chunk(const tq_parquet* pq, int32_t rg, int32_t c, int64_t* file_off, int64_t* bytes,
                           int32_t* codec) {
  if (!pq || rg < 0 || rg >= (int32_t)pq->rgs.size() || c < 0 || c >= (int32_t)pq->cols.size())
    return fail(TQ_EINVAL, "no chunk (%d, %d)", rg, c);
  const PqChunk& ch = pq->rgs[(size_t)rg].chunks[(size_t)c];
  if (file_off) *file_off = ch.start;
  if (bytes) *bytes = ch.bytes;
  if (codec) *codec = ch.codec;
  return TQ_OK;
}

tq_status tq_parquet_preload(tq_parquet* pq, tq_pagepool* pool, int32_t rg0, int32_t rg1, const int32_t* cols,
                             int32_t ncol, int64_t merge_gap, tq_preload** out) {
  if (!out) return fail(TQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pq || !pool) return fail(TQ_EINVAL, "file or pool is NULL");
  if (rg0 < 0 || rg1 > (int32_t)pq->rgs.size() || rg0 > rg1) return fail(TQ_EINVAL, "row groups [%d, %d)", rg0, rg1);
  if (ncol <= 0 || ncol > TQ_MAX_COLS || !cols) return fail(TQ_EINVAL, "column count %d", ncol);
  if (merge_gap < 0) return fail(TQ_EINVAL, "negative merge gap");
  struct Range {
    int64_t off, bytes;
  };
  std::vector<Range> ranges;
  for (int32_t i = 0; i < ncol; i++) {
    const int32_t c = cols[i];
    if (c < 0 || c >= (int32_t)pq->cols.size()) return fail(TQ_EINVAL, "no column %d", c);
    for (int32_t j = 0; j < i; j++)
      if (cols[j] == c) return fail(TQ_EINVAL, "column %d listed twice", c);
    if (!width_of_type(pq->cols[(size_t)c].type))
      return fail(TQ_EINVAL, "column %s: physical type %d is not INT32 or INT64", pq->cols[(size_t)c].name.c_str(),
                  pq->cols[(size_t)c].type);
    for (int32_t g = rg0; g < rg1; g++) {
      const PqChunk& ch = pq->rgs[(size_t)g].chunks[(size_t)c];
      if (ch.codec != 0 && ch.codec != kPqSnappy)
        return fail(TQ_EINVAL, "column %s: codec %d; the decoder takes uncompressed or Snappy chunks",
                    pq->cols[(size_t)c].name.c_str(), ch.codec);
      if (ch.bytes > 0) ranges.push_back(Range{ch.start, ch.bytes});
    }
  }
  // merge ranges whose gap is at most merge_gap (one read instead of several)
  std::sort(ranges.begin(), ranges.end(), [](const Range& a, const Range& b) { return a.off < b.off; });
  std::vector<Range> merged;
  for (const Range& r : ranges) {
    if (!merged.empty() && r.off - (merged.back().off + merged.back().bytes) <= merge_gap)
      merged.back().bytes = std::max(merged.back().bytes, r.off + r.bytes - merged.back().off);
    else
      merged.push_back(r);
  }
  auto* p = new tq_preload();
  p->pq = pq;
  p->pool = pool;
  p->rg0 = rg0;
  p->rg1 = rg1;
  p->cols.assign(cols, cols + ncol);
  for (int32_t g = rg0; g < rg1; g++) p->rows += pq->rgs[(size_t)g].num_rows;
  const size_t pb = tq_pagepool_page_bytes(pool);
  int64_t raw = 0;
  for (const Range& r : merged) {
    tq_parquet_read rd;
    rd.file_off = r.off;
    rd.bytes = r.bytes;
    rd.raw_off = raw;
    const int64_t npages = (int64_t)((r.bytes + pb - 1) / pb);
    rd.pages.resize((size_t)npages);
    if (npages > 0 && tq_pagepool_alloc(pool, npages, rd.pages.data()) != TQ_OK) {
      pq_release_pages(p);
      delete p;
      return fail(TQ_ENOMEM, "the pool has fewer than %lld free pages for a read of %lld bytes", (long long)npages,
                  (long long)r.bytes);
    }
    p->reads.push_back(std::move(rd));
    raw += align256(r.bytes);
  }
  p->raw_bytes = raw;
  for (const tq_parquet_read& r : p->reads)
    for (size_t i = 0; i < r.pages.size(); i++) {
      char* page = static_cast<char*>(tq_pagepool_page(pool, r.pages[i]));
      const int64_t page_end = std::min<int64_t>((int64_t)((i + 1) * pb), r.bytes);
      for (int64_t at = (int64_t)(i * pb); at < page_end; at += kPqReadPiece)
        p->pieces.push_back(tq_parquet_piece{r.file_off + at, std::min(kPqReadPiece, page_end - at),
                                             page + (at - (int64_t)(i * pb))});
    }
  const int nthreads = (int)std::min<int64_t>(kPqReaders, (int64_t)p->pieces.size());
  try {
    for (int t = 0; t < nthreads; t++) p->readers.emplace_back(read_pieces, p);
  } catch (const std::system_error&) {  // no more threads: those started (or this one) read the rest
    if (p->readers.empty()) read_pieces(p);
  }
  *out = p;
  return TQ_OK;
}

int32_t tq_preload_num_reads(const tq_preload* p) { return p ? (int32_t)p->reads.size() : -1; }

tq_status tq_preload_read(const tq_preload* p, int32_t i, int64_t* file_off, int64_t* bytes) {
  if (!p || i < 0 || i >= (int32_t)p->reads.size()) return fail(TQ_EINVAL, "no read %d", i);
  if (file_off) *file_off = p->reads[(size_t)i].file_off;
  if (bytes) *bytes = p->reads[(size_t)i].bytes;
  return TQ_OK;
}

tq_status tq_preload_work_bytes(tq_preload* p, size_t* bytes) {
  if (!p || !bytes) return fail(TQ_EINVAL, "preload or bytes is NULL");
  tq_status s;
  if ((s = pq_join(p))) return s;
  if ((s = pq_parse_pages(p))) return s;
  *bytes = pq_work_bytes(p);
  return TQ_OK;
}

int64_t tq_preload_rows(const tq_preload* p) { return p ? p->rows : -1; }

int64_t tq_preload_num_pages(const tq_preload* p) { return p && p->parsed ? (int64_t)p->pages.size() : -1; }

tq_status tq_preload_page(const tq_preload* p, int64_t i, int64_t* row0, int32_t* nrows, int32_t* col,
                          int32_t* kind, int32_t* encoding) {
  if (!p || !p->parsed || i < 0 || i >= (int64_t)p->pages.size()) return fail(TQ_EINVAL, "no page %lld", (long long)i);
  const PqPage& d = p->pages[(size_t)i];
  if (row0) *row0 = d.row0;
  if (nrows) *nrows = d.nrows;
  if (col) *col = d.col;
  if (kind) *kind = d.kind;
  if (encoding) *encoding = d.encoding;
  return TQ_OK;
}

void tq_preload_free(tq_preload* p) {
  if (!p) return;
  pq_join(p);
  pq_release_pages(p);
  delete p;
}

}  // extern "C"
