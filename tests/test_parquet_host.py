"""Parquet scan, host side (no GPU): the footer against pyarrow's reading of
it, byte ranges and their merging, the page walk's invariants, and the files
the decoder refuses. Files are written by pyarrow from seeded columns."""
import os

import numpy as np
import pytest

pyarrow = pytest.importorskip("pyarrow")
import pyarrow.parquet as pq  # noqa: E402

from paper_2508_05029_amd import tq  # noqa: E402
from tests import pqfiles  # noqa: E402


@pytest.fixture(scope="module")
def small(tmp_path_factory):
    d = tmp_path_factory.mktemp("pq")
    cols = pqfiles.columns(50_000, 7)
    return pqfiles.write(str(d / "small.parquet"), cols, row_group_size=20_000, data_page_size=16_384), cols


def test_footer_matches_pyarrow(small):
    path, cols = small
    f = tq.ParquetFile(path)
    m = pq.ParquetFile(path).metadata
    assert f.num_rows == m.num_rows == 50_000
    assert f.num_row_groups == m.num_row_groups == 3
    assert [f.row_group_rows(i) for i in range(3)] == [m.row_group(i).num_rows for i in range(3)]
    assert f.columns() == [(name, 8 if v.dtype == np.int64 else 4, mask is not None) for name, v, mask, _ in cols]
    for rg in range(3):
        for j in range(len(cols)):
            c = m.row_group(rg).column(j)
            start = c.dictionary_page_offset if c.has_dictionary_page else c.data_page_offset
            assert f.chunk(rg, j) == (start, c.total_compressed_size, 0)


def test_ranges_merge_by_gap(small):
    path, cols = small
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 16, 256, pinned=False)
    # two columns that are not adjacent in the file: separate reads unless the gap allows
    chunks = sorted(f.chunk(rg, c)[:2] for rg in range(3) for c in (0, 3))
    pl = f.preload(pool, 0, 3, [0, 3], merge_gap=0)
    reads = pl.reads()
    assert sum(n for _, n in reads) == sum(n for _, n in chunks)
    assert reads == chunks or len(reads) < len(chunks)
    pl.free()
    big = f.preload(pool, 0, 3, [0, 3], merge_gap=1 << 30)
    assert big.reads() == [(chunks[0][0], chunks[-1][0] + chunks[-1][1] - chunks[0][0])]
    big.free()
    assert pool.free_pages() == 256  # every page back


def test_page_walk_covers_every_row_once(small):
    path, cols = small
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 16, 256, pinned=False)
    sel = list(range(len(cols)))
    pl = f.preload(pool, 0, 3, sel, merge_gap=4096)
    assert pl.rows == 50_000
    assert pl.work_bytes() > 0
    pages = pl.pages()
    m = pq.ParquetFile(path).metadata
    for c in sel:
        data = [(r0, n) for r0, n, col, kind, _ in pages if col == c and kind == 0]
        # data pages tile the rows in order
        assert data[0][0] == 0 and all(a[0] + a[1] == b[0] for a, b in zip(data, data[1:]))
        assert data[-1][0] + data[-1][1] == 50_000
        ndict = sum(1 for _, _, col, kind, _ in pages if col == c and kind == 2)
        assert ndict == sum(m.row_group(rg).column(c).has_dictionary_page for rg in range(3))
        enc = {e for _, _, col, kind, e in pages if col == c and kind == 0}
        assert enc <= ({0, 8} if cols[c][3] else {0})
    # fk's dictionary outgrows its page limit: dictionary pages, then PLAIN ones
    pl.free()


def test_dictionary_fallback_file_has_both_encodings(tmp_path):
    cols = pqfiles.columns(300_000, 9)
    path = pqfiles.write(str(tmp_path / "fb.parquet"), cols, dictionary_pagesize_limit=64 << 10,
                         data_page_size=64 << 10)
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 20, 64, pinned=False)
    pl = f.preload(pool, 0, f.num_row_groups, [2], merge_gap=0)
    pl.work_bytes()
    enc = [e for _, _, _, kind, e in pl.pages() if kind == 0]
    assert 8 in enc and 0 in enc
    pl.free()


def test_version_2_pages_walk(tmp_path):
    cols = pqfiles.columns(30_000, 10)
    path = pqfiles.write(str(tmp_path / "v2.parquet"), cols, version="2.0", data_page_size=8192)
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 16, 64, pinned=False)
    pl = f.preload(pool, 0, 1, list(range(len(cols))), merge_gap=0)
    pl.work_bytes()
    assert sum(n for _, n, _, kind, _ in pl.pages() if kind == 0) == 30_000 * len(cols)
    pl.free()


def test_refused_files(tmp_path):
    cols = pqfiles.columns(1000, 11)
    gz = pqfiles.write(str(tmp_path / "g.parquet"), cols, compression="gzip")
    pool = tq.PagePool(1 << 16, 16, pinned=False)
    f = tq.ParquetFile(gz)
    with pytest.raises(tq.TqError, match="codec"):
        f.preload(pool, 0, 1, [0], merge_gap=0)
    # Snappy chunks are taken (inflated on the GPU)
    sn = tq.ParquetFile(pqfiles.write(str(tmp_path / "s.parquet"), cols, compression="snappy"))
    pl = sn.preload(pool, 0, 1, [0, 1], merge_gap=0)
    assert pl.work_bytes() > 0
    pl.free()
    # strings and nested columns
    pa = pyarrow
    pq.write_table(pa.table({"s": pa.array(["a", "b"])}), str(tmp_path / "str.parquet"), compression="NONE")
    g = tq.ParquetFile(str(tmp_path / "str.parquet"))
    assert g.columns() == [("s", 0, True)]
    with pytest.raises(tq.TqError, match="type"):
        g.preload(pool, 0, 1, [0], merge_gap=0)
    pq.write_table(pa.table({"n": pa.array([{"x": 1}, {"x": 2}])}), str(tmp_path / "nest.parquet"),
                   compression="NONE")
    with pytest.raises(tq.TqError, match="nested"):
        tq.ParquetFile(str(tmp_path / "nest.parquet"))
    # not Parquet, truncated
    bad = tmp_path / "bad.parquet"
    bad.write_bytes(b"PAR1" + b"\0" * 100)
    with pytest.raises(tq.TqError):
        tq.ParquetFile(str(bad))
    raw = open(gz, "rb").read()
    (tmp_path / "cut.parquet").write_bytes(raw[: len(raw) // 2])
    with pytest.raises(tq.TqError):
        tq.ParquetFile(str(tmp_path / "cut.parquet"))
    # argument checks
    f2 = tq.ParquetFile(pqfiles.write(str(tmp_path / "ok.parquet"), cols))
    for rg0, rg1, sel in [(0, 2, [0]), (1, 0, [0]), (0, 1, []), (0, 1, [0, 0]), (0, 1, [99])]:
        with pytest.raises(tq.TqError):
            f2.preload(pool, rg0, rg1, sel, merge_gap=0)
    assert pool.free_pages() == 16


def test_large_pages_are_read_in_pieces(tmp_path):
    """Pool pages of 8 MiB are read as 2 MiB pieces by several threads: with a
    page header every 64 KiB, a piece left unread breaks the walk."""
    cols = pqfiles.columns(600_000, 13)
    path = pqfiles.write(str(tmp_path / "big.parquet"), cols, data_page_size=65_536)
    f = tq.ParquetFile(path)
    pool = tq.PagePool(8 << 20, 8, pinned=False)
    sel = list(range(len(cols)))
    pl = f.preload(pool, 0, f.num_row_groups, sel, merge_gap=1 << 20)
    assert sum(n for _, n in pl.reads()) > 4 << 20  # several pieces per page
    assert pl.work_bytes() > 0
    pages = pl.pages()
    for c in sel:
        data = [(r0, n) for r0, n, col, kind, _ in pages if col == c and kind == 0]
        assert data[0][0] == 0 and all(a[0] + a[1] == b[0] for a, b in zip(data, data[1:]))
        assert data[-1][0] + data[-1][1] == 600_000
    pl.free()
    assert pool.free_pages() == 8


def test_file_cut_after_open_fails_the_read(tmp_path):
    cols = pqfiles.columns(200_000, 14)
    path = pqfiles.write(str(tmp_path / "cut.parquet"), cols, data_page_size=65_536)
    f = tq.ParquetFile(path)  # footer read while the file is whole
    os.truncate(path, os.path.getsize(path) // 3)
    pool = tq.PagePool(1 << 20, 16, pinned=False)
    pl = f.preload(pool, 0, f.num_row_groups, list(range(len(cols))), merge_gap=1 << 20)
    with pytest.raises(tq.TqError, match="reading"):
        pl.work_bytes()
    pl.free()
    assert pool.free_pages() == 16


def test_pool_too_small_is_refused(small):
    path, _ = small
    f = tq.ParquetFile(path)
    pool = tq.PagePool(4096, 4, pinned=False)
    with pytest.raises(tq.TqError) as e:
        f.preload(pool, 0, 3, [0], merge_gap=0)
    assert e.value.status == tq.TQ_ENOMEM
    assert pool.free_pages() == 4


def test_hand_written_file_is_valid_parquet_and_walks(tmp_path):
    """The tests' own minimal writer (Snappy elements placed by hand): pyarrow
    reads the file back, and the host side finds its one chunk and page."""
    from tests import pqhand as H
    rng = np.random.default_rng(5)
    raw = rng.integers(0, 256, 70_000 + 8 * 10).astype(np.uint8).tobytes()[:70_000]
    out = bytearray(raw)
    els = [H.literal(raw)]
    for off, ln in [(68_000, 64), (1, 16)]:
        for _ in range(ln):
            out.append(out[len(out) - off])
        els.append(H.copy(off, ln))
    n = len(out) // 8
    body = H.snappy_block(els, len(out))
    path = H.write(str(tmp_path / "h.parquet"), [body], [n])
    assert np.array(pq.read_table(path)["x"]).tobytes() == bytes(out)
    f = tq.ParquetFile(path)
    assert f.columns() == [("x", 8, False)] and f.num_rows == n
    assert f.chunk(0, 0)[2] == 1  # Snappy
    pool = tq.PagePool(1 << 20, 8, pinned=False)
    pl = f.preload(pool, 0, 1, [0], merge_gap=0)
    pl.work_bytes()
    assert pl.pages() == [(0, n, 0, 0, 0)]
    pl.free()
