"""GPU: host -> device streaming from the page pool, and the out-of-core
partitioned join + aggregate under budgets that do and do not force spills,
against the CPU oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402
from paper_2508_05029_amd.hosttable import HostTable  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("pinned", [True, False])
def test_stream_delivers_every_batch_byte_exact(pinned):
    """Each staged batch is copied out by a filter_project with identity
    expressions; the concatenation must equal the host columns."""
    pool = tq.PagePool(8192, 600, pinned=pinned)
    n, rpb = 20_011, 1_777
    rng = np.random.default_rng(1)
    cols = {"a": rng.integers(-2**62, 2**62, n).astype(np.int64), "b": rng.integers(-2**31, 2**31, n).astype(np.int32),
            "c": rng.integers(0, 256, n).astype(np.uint8)}
    t = HostTable(pool, [("a", np.int64), ("b", np.int32), ("c", np.uint8)], n, rpb)
    t.fill_numpy(cols)
    staging = torch.empty(3 * t.max_batch_bytes(), dtype=torch.uint8, device="cuda")
    outs = [torch.empty(n, dtype=torch.int64, device="cuda") for _ in range(3)]
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    scratch = torch.empty(tq.filter_project_scratch_bytes(rpb), dtype=torch.uint8, device="cuda")
    starts = [b[0] for b in t.batches]

    def on_batch(i, dcols, nrows, stream):
        base = starts[i]
        views = [o[base:base + nrows] for o in outs]
        # device columns arrive as raw pointers: wrap them as tq columns
        c = (tq.Col * 3)(*[tq.Col(p, ty) for p, ty in dcols])
        e = tq.exprs([[(j, 1, 0)] for j in range(3)])
        import ctypes
        outp = (ctypes.c_void_p * 3)(*[v.data_ptr() for v in views])
        st = tq.lib().tq_filter_project(c, 3, nrows, None, 0, e, 3, outp, None, cnt.data_ptr(), scratch.data_ptr(),
                                        scratch.numel(), stream)
        return st

    side = torch.cuda.Stream()
    tq.pagepool_stream(pool, t.c_batches(), staging, 3, on_batch, side, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for j, k in enumerate("abc"):
        assert outs[j].cpu().numpy().tolist() == cols[k].astype(np.int64).tolist()
    t.free()
    pool.close()


def _ooc_tables(pool, n_dim, n_fact, rows_per_batch, seed):
    d, f = wl.ooc_tables_numpy(n_fact, n_dim, seed)
    dt = HostTable(pool, wl.OOC_DIM_COLS, n_dim, rows_per_batch)
    dt.fill_numpy(d)
    ft = HostTable(pool, wl.OOC_FACT_COLS, n_fact, rows_per_batch)
    ft.fill_numpy(f)
    return d, f, dt, ft


@pytest.mark.parametrize("budget_mb,bits,keep_all", [(64, 4, True), (16, 4, True), (64, 6, False), (14, 6, False),
                                                    (64, 0, True)])
def test_ooc_join_agg_matches_oracle(budget_mb, bits, keep_all):
    say(f"ooc budget={budget_mb}MB bits={bits} keep_all={keep_all}")
    pool = tq.PagePool(256 << 10, 2000, pinned=True)
    d, f, dt, ft = _ooc_tables(pool, 100_000, 600_000, 50_000, seed=31)
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg(d, f, q)
    job = pipeline.OocJoinAgg(q, dt, ft, budget_mb << 20, log2_fanout=bits, chunk_bytes=64 << 10, keep_all=keep_all,
                              exchange="partitioned")
    st = job.run()
    got = job.result()
    say(st.as_dict())
    assert got["join_rows"] == want["join_rows"]
    assert got["keys"].tolist() == want["keys"].tolist()
    assert got["count"].tolist() == want["count"].tolist()
    assert got["sums"].tolist() == want["sums"].tolist()
    assert st.fact_rows == 600_000
    assert st.dim_rows_kept == int(((d["date"] >= 730) & (d["date"] <= 1094)).sum())
    assert st.peak_budget_bytes <= budget_mb << 20
    assert st.exchange == tq.TQ_EXCHANGE_PARTITIONED and st.dim_restreams == 0 and st.est_dim_rows == 0
    if budget_mb <= 16:
        assert st.spilled_chunks > 0 and st.reloaded_chunks > 0  # the budget forced spilling
    else:
        assert st.spilled_chunks == 0
    assert job.budget.used == 0  # every reservation was released
    dt.free()
    ft.free()
    assert pool.free_pages() == 2000  # spill pages were returned too
    pool.close()


def test_ooc_budget_too_small_fails_cleanly():
    pool = tq.PagePool(256 << 10, 600, pinned=True)
    d, f, dt, ft = _ooc_tables(pool, 10_000, 50_000, 20_000, seed=5)
    job = pipeline.OocJoinAgg(wl.JOIN_AGG_QUERY, dt, ft, 1 << 20, log2_fanout=2, chunk_bytes=64 << 10)
    with pytest.raises(tq.TqError) as e:
        job.run()
    assert e.value.status == tq.TQ_ENOMEM
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 600
    pool.close()


def _check_result(job, d, f, q):
    want = oracle.join_agg(d, f, q)
    got = job.result()
    assert got["join_rows"] == want["join_rows"]
    assert got["keys"].tolist() == want["keys"].tolist()
    assert got["count"].tolist() == want["count"].tolist()
    assert got["sums"].tolist() == want["sums"].tolist()


def _kept(d):
    return int(((d["date"] >= 730) & (d["date"] <= 1094)).sum())


@pytest.mark.parametrize("bits,keep_all", [(4, True), (0, False)])
def test_ooc_adaptive_exchange_chooses_one_table(bits, keep_all):
    """A filtered dimension that fits the budget: the Adaptive Exchange takes
    one table, the fact side is probed as it streams (nothing spilled or
    reloaded), and the estimate from the first batches is close."""
    say(f"ooc adaptive single bits={bits} keep_all={keep_all}")
    pool = tq.PagePool(256 << 10, 2000, pinned=True)
    d, f, dt, ft = _ooc_tables(pool, 100_000, 600_000, 10_000, seed=37)
    q = wl.JOIN_AGG_QUERY
    job = pipeline.OocJoinAgg(q, dt, ft, 64 << 20, log2_fanout=bits, chunk_bytes=64 << 10, keep_all=keep_all)
    st = job.run()
    say(st.as_dict())
    _check_result(job, d, f, q)
    assert st.exchange == tq.TQ_EXCHANGE_SINGLE and st.dim_restreams == 0
    assert st.spilled_chunks == 0 and st.reloaded_chunks == 0 and st.bytes_d2h == 0
    assert st.dim_rows_kept == _kept(d) and st.fact_rows == 600_000
    # decided after the first batches holding an eighth of the rows (10K-row batches: two of ten)
    assert st.est_from_rows == 20_000
    assert abs(st.est_dim_rows - _kept(d)) <= 0.1 * _kept(d)
    assert st.peak_budget_bytes <= 64 << 20
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 2000
    pool.close()


def test_ooc_adaptive_exchange_partitions_when_one_table_does_not_fit():
    say("ooc adaptive partitioned")
    pool = tq.PagePool(256 << 10, 3000, pinned=True)
    d, f, dt, ft = _ooc_tables(pool, 1_000_000, 600_000, 50_000, seed=41)
    q = wl.JOIN_AGG_QUERY
    job = pipeline.OocJoinAgg(q, dt, ft, 16 << 20, log2_fanout=4, chunk_bytes=64 << 10)
    st = job.run()
    say(st.as_dict())
    _check_result(job, d, f, q)
    assert st.exchange == tq.TQ_EXCHANGE_PARTITIONED and st.dim_restreams == 0
    assert st.est_from_rows == 150_000 and abs(st.est_dim_rows - _kept(d)) <= 0.1 * _kept(d)
    assert st.spilled_chunks > 0 and st.peak_budget_bytes <= 16 << 20
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 3000
    pool.close()


def test_ooc_adaptive_exchange_restreams_after_a_low_estimate():
    """Dimension rows sorted by date: the first batches keep nothing, the
    estimate says one table, and the exact count at the end of the dimension
    side does not fit, so the dimension is streamed again and partitioned."""
    say("ooc adaptive restream")
    pool = tq.PagePool(256 << 10, 3000, pinned=True)
    d, f = wl.ooc_tables_numpy(600_000, 1_000_000, 43)
    order = np.argsort(d["date"], kind="stable")
    d = {k: v[order] for k, v in d.items()}
    dt = HostTable(pool, wl.OOC_DIM_COLS, 1_000_000, 50_000)
    dt.fill_numpy(d)
    ft = HostTable(pool, wl.OOC_FACT_COLS, 600_000, 50_000)
    ft.fill_numpy(f)
    q = wl.JOIN_AGG_QUERY
    job = pipeline.OocJoinAgg(q, dt, ft, 16 << 20, log2_fanout=4, chunk_bytes=64 << 10)
    st = job.run()
    say(st.as_dict())
    _check_result(job, d, f, q)
    assert st.est_dim_rows == 0 and st.est_from_rows == 150_000
    assert st.exchange == tq.TQ_EXCHANGE_PARTITIONED and st.dim_restreams == 1
    assert st.dim_rows_kept == _kept(d)
    assert st.peak_budget_bytes <= 16 << 20
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 3000
    pool.close()


def test_ooc_forced_single_table_that_does_not_fit_fails_cleanly():
    pool = tq.PagePool(256 << 10, 3000, pinned=True)
    d, f, dt, ft = _ooc_tables(pool, 1_000_000, 100_000, 50_000, seed=47)
    job = pipeline.OocJoinAgg(wl.JOIN_AGG_QUERY, dt, ft, 16 << 20, log2_fanout=4, chunk_bytes=64 << 10, exchange="single")
    with pytest.raises(tq.TqError) as e:
        job.run()
    assert e.value.status == tq.TQ_ENOMEM
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 3000
    pool.close()


@pytest.mark.parametrize("exchange", ["auto", "partitioned"])
def test_ooc_dimension_filter_keeps_nothing(exchange):
    """No dimension row passes the filter: both exchanges produce no group."""
    say(f"ooc empty dimension side, exchange={exchange}")
    pool = tq.PagePool(256 << 10, 1000, pinned=True)
    d, f = wl.ooc_tables_numpy(200_000, 50_000, 53)
    d["date"][:] = 5  # outside the query's window
    dt = HostTable(pool, wl.OOC_DIM_COLS, 50_000, 20_000)
    dt.fill_numpy(d)
    ft = HostTable(pool, wl.OOC_FACT_COLS, 200_000, 20_000)
    ft.fill_numpy(f)
    q = wl.JOIN_AGG_QUERY
    job = pipeline.OocJoinAgg(q, dt, ft, 32 << 20, log2_fanout=4, chunk_bytes=64 << 10, exchange=exchange)
    st = job.run()
    got = job.result()
    assert st.dim_rows_kept == 0 and st.fact_rows == 200_000
    assert got["join_rows"] == 0 and len(got["count"]) == 0
    assert st.exchange == (tq.TQ_EXCHANGE_SINGLE if exchange == "auto" else tq.TQ_EXCHANGE_PARTITIONED)
    assert job.budget.used == 0
    dt.free()
    ft.free()
    assert pool.free_pages() == 1000
    pool.close()
