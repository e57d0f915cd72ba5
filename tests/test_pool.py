"""Page pool, batch layout, host tables and the budget, on the CPU (pageable pool)."""
import numpy as np
import pytest

from paper_2508_05029_amd import tq
from paper_2508_05029_amd.hosttable import HostTable


def test_pool_alloc_free_all_or_nothing():
    p = tq.PagePool(4096, 10, pinned=False)
    a = p.alloc(6)
    assert len(set(a)) == 6 and p.free_pages() == 4
    with pytest.raises(tq.TqError) as e:
        p.alloc(5)  # all or nothing
    assert e.value.status == tq.TQ_ENOMEM and p.free_pages() == 4
    b = p.alloc(4)
    assert p.free_pages() == 0 and not set(a) & set(b)
    p.free(a)
    assert p.free_pages() == 6
    addrs = {p.page(i) for i in range(10)}
    assert len(addrs) == 10 and all(x % 4096 == 0 for x in addrs)
    assert p.page(10) == 0 and p.page(-1) == 0
    p.close()


def test_pool_rejects_bad_sizes():
    with pytest.raises(tq.TqError):
        tq.PagePool(1000, 4, pinned=False)  # not a multiple of 256
    with pytest.raises(tq.TqError):
        tq.PagePool(4096, 0, pinned=False)


def test_batch_layout_aligns_and_counts_pages():
    offs, nbytes, npages = tq.batch_layout(1000, [tq.TQ_I64, tq.TQ_I32, tq.TQ_U8, tq.TQ_I64], 4096)
    assert offs == [0, 8192, 12288, 13312]
    assert nbytes == 13312 + 8000 and npages == (nbytes + 4095) // 4096
    assert all(o % 256 == 0 for o in offs)


@pytest.mark.parametrize("rows_per_batch", [1, 333, 1000, 5000])
def test_host_table_round_trip_across_page_boundaries(rows_per_batch):
    pool = tq.PagePool(1024, 4000, pinned=False)
    rng = np.random.default_rng(rows_per_batch)
    n = 3001
    cols = {"a": rng.integers(-2**62, 2**62, n).astype(np.int64), "b": rng.integers(-2**31, 2**31, n).astype(np.int32),
            "c": rng.integers(0, 256, n).astype(np.uint8)}
    t = HostTable(pool, [("a", np.int64), ("b", np.int32), ("c", np.uint8)], n, rows_per_batch)
    t.fill_numpy(cols)
    for k, v in cols.items():
        assert (t.read_column(k) == v).all()
    # some column of some batch straddles a page
    assert any(len(list(t.pieces(b, 0))) > 1 for b in range(len(t.batches))) or rows_per_batch < 200
    t.free()
    assert pool.free_pages() == 4000


def test_host_table_frees_pages_when_the_pool_runs_out():
    pool = tq.PagePool(1024, 5, pinned=False)
    with pytest.raises(tq.TqError):
        HostTable(pool, [("a", np.int64)], 10_000, 100)
    assert pool.free_pages() == 5


def test_budget_reservations():
    b = tq.Budget(1000)
    b.reserve(600)
    assert not b.try_reserve(500)  # would exceed the cap: the caller spills and retries
    b.reserve(400)
    assert b.used == 1000 and b.peak == 1000
    b.release(700)
    assert b.used == 300 and b.peak == 1000
    b.release(10_000)  # never below zero
    assert b.used == 0 and b.cap == 1000


def test_ooc_rejects_bad_plans_before_any_work():
    """tq_ooc_join_agg validates the plan before it touches a device: an
    unknown exchange mode, a fan-out past 2^10 and a single staging slot all
    return TQ_EINVAL (the work and state pointers are never dereferenced)."""
    import ctypes
    fake = 0x100000
    pool = tq.PagePool(1 << 16, 16, pinned=False)
    rng = np.random.default_rng(3)
    dt = HostTable(pool, [("key", np.int64), ("group", np.int32), ("date", np.int32)], 100, 50)
    dt.fill_numpy({"key": np.arange(100, dtype=np.int64), "group": rng.integers(0, 5, 100).astype(np.int32),
                   "date": rng.integers(0, 2000, 100).astype(np.int32)})
    ft = HostTable(pool, [("fk", np.int64), ("price", np.int64)], 100, 50)
    ft.fill_numpy({"fk": rng.integers(0, 100, 100).astype(np.int64), "price": np.arange(100, dtype=np.int64)})
    preds = tq.preds([(2, 730, 1094)])
    sums = tq.exprs([[(1, 1, 0)]])
    d_arr, d_keep = dt.c_batches()
    f_arr, f_keep = ft.c_batches()
    budget = tq.Budget(1 << 24)
    L = tq._bind_more()

    def run(**over):
        kw = dict(log2_fanout=2, nslots=2, exchange=tq.TQ_EXCHANGE_AUTO)
        kw.update(over)
        plan = tq.OocPlan(0, 1, ctypes.cast(preds, ctypes.POINTER(tq.PredS)), 1, 0, 3,
                          ctypes.cast(sums, ctypes.POINTER(tq.ExprS)), 1, 5, kw["log2_fanout"], 0.5, 0, 1 << 16,
                          kw["nslots"], kw["exchange"])
        st = tq.OocStats()
        return L.tq_ooc_join_agg(pool.h, d_arr, len(dt.batches), f_arr, len(ft.batches), ctypes.byref(plan),
                                 budget.h, fake, 1 << 24, fake, ctypes.byref(st), None, None)

    assert run(exchange=3) == tq.TQ_EINVAL
    assert run(exchange=-1) == tq.TQ_EINVAL
    assert run(log2_fanout=11) == tq.TQ_EINVAL
    assert run(nslots=1) == tq.TQ_EINVAL
    assert budget.used == 0
    dt.free()
    ft.free()
    pool.close()
