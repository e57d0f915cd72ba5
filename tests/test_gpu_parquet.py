"""GPU: Parquet pages decoded by the scan kernels equal the columns pyarrow
wrote (values bit-exact, NULL rows 0, validity bits exact): PLAIN and
dictionary pages, a dictionary that falls back to PLAIN, data pages v1 and
v2, optional columns with NULLs (none, some, all), several row groups and
pages, column and row-group subsets; then a join + aggregate over decoded
columns against the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
pytest.importorskip("pyarrow")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402
from tests import pqfiles  # noqa: E402

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def decode(path, sel, rg0=None, rg1=None, page_bytes=1 << 20, merge_gap=1 << 20, valid_for_all=False):
    f = tq.ParquetFile(path)
    rg0 = 0 if rg0 is None else rg0
    rg1 = f.num_row_groups if rg1 is None else rg1
    pool = tq.PagePool(page_bytes, 512)
    pl = f.preload(pool, rg0, rg1, sel, merge_gap=merge_gap)
    n = pl.rows
    work = torch.empty(pl.work_bytes(), dtype=torch.uint8, device=DEV)
    meta = f.columns()
    outs = []
    for c in sel:
        _, t, nullable = meta[c]
        data = torch.full((max(n, 1),), -1, dtype=torch.int64 if t == 8 else torch.int32, device=DEV)
        valid = (torch.full((((n + 31) // 32) * 4 or 4,), 0xAB, dtype=torch.uint8, device=DEV)
                 if nullable or valid_for_all else None)
        outs.append((data, valid))
    pl.decode(work, outs)
    tq.check(work)
    pl.free()
    assert pool.free_pages() == 512
    res = []
    for data, valid in outs:
        v = data[:n].cpu().numpy()
        bits = None if valid is None else np.unpackbits(valid.cpu().numpy(), bitorder="little")[:n].astype(bool)
        res.append((v, bits))
    return res, n


def expect(cols, c, lo, hi):
    name, vals, mask, _ = cols[c]
    v = vals[lo:hi]
    m = np.ones(hi - lo, bool) if mask is None else mask[lo:hi]
    return np.where(m, v, 0), m


def check(cols, sel, res, lo, hi):
    for c, (v, bits) in zip(sel, res):
        want, m = expect(cols, c, lo, hi)
        assert v.tolist() == want.tolist(), cols[c][0]
        if bits is not None:
            assert bits.tolist() == m.tolist(), cols[c][0]


@pytest.mark.parametrize("n,rg,page,version,codec", [(50_000, 20_000, 16_384, "1.0", "NONE"),
                                                     (50_000, 20_000, 8_192, "2.0", "NONE"),
                                                     (1, None, None, "1.0", "NONE"), (1025, 1024, 512, "1.0", "NONE"),
                                                     (300_000, None, 1 << 20, "1.0", "NONE"),
                                                     (50_000, 20_000, 16_384, "1.0", "snappy"),
                                                     (50_000, 20_000, 8_192, "2.0", "snappy"),
                                                     (1, None, None, "1.0", "snappy"),
                                                     (300_000, None, 1 << 20, "1.0", "snappy")])
def test_decode_matches_written_columns(tmp_path, n, rg, page, version, codec):
    say(f"parquet decode n={n} rg={rg} page={page} v{version} {codec}")
    cols = pqfiles.columns(n, 21)
    path = pqfiles.write(str(tmp_path / "t.parquet"), cols, row_group_size=rg, data_page_size=page, version=version,
                         compression=codec)
    sel = list(range(len(cols)))
    res, rows = decode(path, sel)
    assert rows == n
    check(cols, sel, res, 0, n)


def test_dictionary_falling_back_to_plain(tmp_path):
    cols = pqfiles.columns(400_000, 22)
    path = pqfiles.write(str(tmp_path / "fb.parquet"), cols, dictionary_pagesize_limit=64 << 10,
                         data_page_size=64 << 10)
    res, n = decode(path, [2, 1])
    check(cols, [2, 1], res, 0, n)


def test_column_and_row_group_subsets(tmp_path):
    cols = pqfiles.columns(100_000, 23)
    path = pqfiles.write(str(tmp_path / "sub.parquet"), cols, row_group_size=30_000, data_page_size=32_768)
    res, n = decode(path, [4, 0], rg0=1, rg1=3, merge_gap=0)
    assert n == 60_000
    check(cols, [4, 0], res, 30_000, 90_000)


def test_required_column_with_a_bitmap_gets_all_ones(tmp_path):
    cols = pqfiles.columns(5000, 24)
    path = pqfiles.write(str(tmp_path / "req.parquet"), cols)
    res, n = decode(path, [0, 3], valid_for_all=True)
    for v, bits in res:
        assert bits.all()
    check(cols, [0, 3], res, 0, n)


def test_scan_then_join_aggregate(tmp_path):
    """The join + aggregate workload's tables, written to Parquet and scanned
    back, feed the join: its result equals the oracle's on the original tables."""
    nd, nf = 150_000, 600_000
    dim, fact = wl.join_agg_tables(nd, nf, seed=25)
    dcols = [(k, v, None, k == "group") for k, v in dim.items()]
    fcols = [(k, v, None, k == "disc") for k, v in fact.items()]
    dpath = pqfiles.write(str(tmp_path / "dim.parquet"), dcols, data_page_size=1 << 20)
    fpath = pqfiles.write(str(tmp_path / "fact.parquet"), fcols, data_page_size=1 << 20)
    dres, _ = decode(dpath, list(range(len(dcols))))
    fres, _ = decode(fpath, list(range(len(fcols))))
    ddev = {k: torch.from_numpy(v).to(DEV) for (k, _, _, _), (v, _) in zip(dcols, dres)}
    fdev = {k: torch.from_numpy(v).to(DEV) for (k, _, _, _), (v, _) in zip(fcols, fres)}
    q = wl.JOIN_AGG_QUERY
    ja = pipeline.JoinAgg(q, nd, 0.5)
    ja.run(ddev, fdev)
    got = ja.result()
    want = oracle.join_agg(dim, fact, q)
    assert got["keys"].tolist() == want["keys"].tolist()
    assert got["count"].tolist() == want["count"].tolist()
    assert got["sums"].tolist() == want["sums"].tolist()


def test_decode_rejects_bad_outputs(tmp_path):
    cols = pqfiles.columns(1000, 26)
    path = pqfiles.write(str(tmp_path / "o.parquet"), cols)
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 16, 64)
    pl = f.preload(pool, 0, 1, [1], merge_gap=0)
    work = torch.empty(pl.work_bytes(), dtype=torch.uint8, device=DEV)
    data = torch.empty(1000, dtype=torch.int64, device=DEV)  # the column is INT32
    with pytest.raises(tq.TqError):
        pl.decode(work, [(data, torch.zeros(128, dtype=torch.uint8, device=DEV))])
    data32 = torch.empty(1000, dtype=torch.int32, device=DEV)
    with pytest.raises(tq.TqError, match="bitmap"):
        pl.decode(work, [(data32, None)])  # nullable column without a bitmap
    with pytest.raises(tq.TqError, match="work buffer"):
        pl.decode(work[:256], [(data32, torch.zeros(128, dtype=torch.uint8, device=DEV))])
    pl.free()
    assert pool.free_pages() == 64


def test_snappy_repeats_and_runs(tmp_path):
    """Snappy bodies of 4 MiB pages with copies of every length class and
    overlapping copies (runs of one value): a column of repeated blocks with
    short repeats, a long run, and a constant column. (The reference
    compressor never copies from further back than 64 KiB or across a 64 KiB
    fragment; the hand-built pages below do.)"""
    n = 400_000
    block = pqfiles.uniform(20_000, -2 ** 62, 2 ** 62, np.int64, 27, 0)
    vals = np.concatenate([block] * (n // 20_000))
    vals[::7] = 5  # short repeats
    vals[1000:9000] = 0  # a long run
    cols = [("rep", vals, None, False), ("run", np.full(n, 3, np.int64), None, False)]
    path = pqfiles.write(str(tmp_path / "rep.parquet"), cols, data_page_size=4 << 20, compression="snappy")
    res, rows = decode(path, [0, 1])
    check(cols, [0, 1], res, 0, rows)


@pytest.mark.parametrize("codec,streams", [("NONE", 4), ("snappy", 4), ("snappy", 1), ("snappy", 2)])
def test_pipelined_row_groups_equal_the_whole_read(tmp_path, codec, streams):
    """read_pipelined (each row group decoded into its slice of one set of
    columns while the next one's bytes are read, successive row groups on
    `streams` streams in turn) equals what pyarrow wrote, also when read twice."""
    cols = pqfiles.columns(100_000, 28)
    path = pqfiles.write(str(tmp_path / "pipe.parquet"), cols, row_group_size=20_000, data_page_size=32_768,
                         compression=codec)
    pool = tq.PagePool(1 << 20, 64)
    names = [c[0] for c in cols]
    scan = pipeline.ParquetScan(path, names, pool, pipe_streams=streams)
    scan.read_pipelined()
    data, valid = scan.read_pipelined()
    scan.check()
    for c, name in enumerate(names):
        want, m = expect(cols, c, 0, 100_000)
        assert data[name].cpu().numpy().tolist() == want.tolist(), name
        if valid[name] is not None:
            bits = np.unpackbits(valid[name].cpu().numpy(), bitorder="little")[:100_000].astype(bool)
            assert bits.tolist() == m.tolist(), name
    assert pool.free_pages() == 64


# ---------------------------------------------------------------------------
# Snappy bodies built element by element (tests/pqhand.py), for the paths the
# reference compressor never takes; pyarrow reads every well-formed one back.

def _hand_page(seed, plan):
    """plan: a list of ('lit', n) / ('copy', offset, length); returns (body, values)."""
    from tests import pqhand as H
    rng = np.random.default_rng(seed)
    out, els = bytearray(), []
    for step in plan:
        if step[0] == "lit":
            b = rng.integers(0, 256, step[1]).astype(np.uint8).tobytes()
            out += b
            els.append(H.literal(b))
        else:
            _, off, ln = step
            for _ in range(ln):
                out.append(out[len(out) - off])
            els.append(H.copy(off, ln))
    pad = (-len(out)) % 8
    if pad:
        out += bytes(pad)
        els.append(H.literal(bytes(pad)))
    return H.snappy_block(els, len(out)), np.frombuffer(bytes(out), np.int64).copy()


@pytest.mark.parametrize("name,plan", [
    # many copies 4000 bytes back, some reaching over a 64 KiB boundary: the in-order pass
    ("back_4000", [("lit", 70_000), ("copy", 9, 64), ("copy", 1, 50)] + [("lit", 30), ("copy", 4000, 64)] * 900),
    # elements aligned with the 64 KiB fragments, copies inside them: the fragment pass
    ("aligned", [("lit", 65_536), ("lit", 30), ("copy", 20, 64)] + [("lit", 34), ("copy", 100, 64)] * 1000),
    # copies from further back than 64 KiB (4-byte offsets): the in-order pass, read from memory
    ("far", [("lit", 70_000), ("copy", 68_000, 64), ("copy", 65_536, 40), ("copy", 1, 64), ("copy", 3, 17)]),
    # a literal across the 64 KiB boundary, then copies reaching back over it
    ("across", [("lit", 65_530), ("lit", 20), ("copy", 30, 64), ("lit", 80_000), ("copy", 70_000, 10)]),
    # literals of about a chain-scan block (960 input bytes) or two, each followed by short
    # elements, so that chains leave blocks at every offset and skip whole blocks: one fragment
    ("block_edges", [e for k in range(40) for e in (("lit", 950 + (k * 7) % 30 + 960 * (k % 2)), ("copy", 8, 40 + k % 25),
                                                     ("lit", 1 + k % 3), ("copy", 1 + k % 5, 64))]),
    # a last fragment of 88 bytes after one that a single literal fills: one batch each
    ("tail_fragment", [("lit", 65_536), ("lit", 16), ("copy", 8, 64), ("copy", 3, 7)]),
    # three fragments that are one literal each, then five bytes
    ("literal_fragments", [("lit", 65_536)] * 3 + [("lit", 5)]),
])
def test_hand_built_snappy_pages(tmp_path, name, plan):
    import pyarrow.parquet as pq
    from tests import pqhand as H
    say(f"hand-built snappy page: {name}")
    body, vals = _hand_page(31, plan)
    path = H.write(str(tmp_path / f"{name}.parquet"), [body], [len(vals)])
    assert np.array(pq.read_table(path)["x"]).tolist() == vals.tolist()  # valid Parquet and Snappy
    res, n = decode(path, [0])
    assert n == len(vals)
    assert res[0][0].tolist() == vals.tolist()


@pytest.mark.parametrize("bad", ["offset_past_start", "length_mismatch", "truncated", "copy_past_end"])
def test_malformed_snappy_bodies_are_reported(tmp_path, bad):
    """A malformed body latches TQ_EINVAL in the work buffer (every access
    stays inside the page's areas); the pool pages come back."""
    from tests import pqhand as H
    body, vals = _hand_page(32, [("lit", 1000), ("copy", 8, 64), ("lit", 2000)])
    n = len(vals)
    if bad == "offset_past_start":
        body = H.snappy_block([H.literal(bytes(16)), H.copy(5000, 8)], n * 8)
    elif bad == "length_mismatch":
        body = H._varint(n * 8 + 8) + body[len(H._varint(n * 8)):]
    elif bad == "truncated":
        body = body[:-500]
    else:
        body = H.snappy_block([H.literal(bytes(16)), H.copy(8, 64)] * 200, n * 8)  # writes past the length
    path = H.write(str(tmp_path / f"{bad}.parquet"), [body], [n])
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 20, 16)
    pl = f.preload(pool, 0, 1, [0], merge_gap=0)
    work = torch.empty(pl.work_bytes(), dtype=torch.uint8, device=DEV)
    data = torch.empty(n, dtype=torch.int64, device=DEV)
    pl.decode(work, [(data, None)])
    with pytest.raises(tq.TqError) as e:
        tq.check(work)
    assert e.value.status == tq.TQ_EINVAL
    pl.free()
    assert pool.free_pages() == 16


def test_a_preload_is_decoded_once(tmp_path):
    cols = pqfiles.columns(2000, 29)
    path = pqfiles.write(str(tmp_path / "once.parquet"), cols)
    f = tq.ParquetFile(path)
    pool = tq.PagePool(1 << 16, 32)
    pl = f.preload(pool, 0, 1, [0], merge_gap=0)
    work = torch.empty(pl.work_bytes(), dtype=torch.uint8, device=DEV)
    data = torch.empty(2000, dtype=torch.int64, device=DEV)
    pl.decode(work, [(data, None)])
    tq.check(work)
    assert pool.free_pages() == 32  # the pages are back already
    with pytest.raises(tq.TqError, match="decoded already"):
        pl.decode(work, [(data, None)])
    pl.free()
    assert data.cpu().numpy().tolist() == cols[0][1].tolist()
