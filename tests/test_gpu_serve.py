"""GPU: the serving loop. Every request's result is the same alone (one
worker, one request at a time) and in the mix (several workers, requests
overlapping on the device), and equals the oracle; admission respects the
budget."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected(setup, q):
    if q.shape == 0:
        t = {k: v[q.fact_first:q.fact_first + q.n_fact] for k, v in setup.fg.items()}
        return oracle.filter_groupby(t, setup.q0)
    d = {k: v[q.dim_first:q.dim_first + q.n_dim] for k, v in setup.dim.items()}
    if q.shape == 1:
        f = {k: v[q.fact_first:q.fact_first + q.n_fact] for k, v in setup.fact.items()}
    else:
        lo = setup.host.batches[q.fact_first][0]
        last = setup.host.batches[q.fact_first + q.n_fact - 1]
        f = {k: v[lo:last[0] + last[1]] for k, v in setup.hfact.items()}
    return oracle.join_agg(d, f, setup.q1)


def packed(setup, q, res, keys, count, sums, i):
    g = res[i].ngroups
    nsum = 5 if q.shape == 0 else 1
    k = keys[i, :g]
    if q.shape == 0:  # the packed key flagA * 2 + flagB
        k = np.stack([k // 2, k % 2], axis=1)
    else:
        k = k.reshape(-1, 1)
    return k, count[i, :g], sums[i, :g, :nsum]


@pytest.fixture(scope="module")
def setup():
    pool = tq.PagePool(1 << 20, 200, pinned=True)
    s = pipeline.ServingSetup(n0=300_000, n_dim=120_000, n1=400_000, n2=400_000, batch_rows=16_384, pool=pool)
    yield s
    s.host.free()
    pool.close()


def test_alone_equals_mix_equals_oracle(setup):
    reqs = wl.serving_requests(40, qps=2000.0, fact_lo=3.0, fact_hi=5.5, seed=wl.SERVE_SEED + 1)
    R = setup.requests(reqs)
    budget = tq.Budget(256 << 20)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    alone = tq.serve_run(setup.T, R, 1, budget, arena, 25)
    mixed = tq.serve_run(setup.T, R, 6, budget, arena, 25)
    assert budget.used == 0
    workers_used = {mixed[0][i].worker for i in range(len(reqs))}
    say(f"workers used in the mix: {sorted(workers_used)}")
    assert len(workers_used) > 1
    bad = []
    for i in range(len(reqs)):
        q = R[i]
        w = expected(setup, q)
        for name, run in (("alone", alone), ("mix", mixed)):
            k, c, sm = packed(setup, q, *run, i)
            if not (k.tolist() == w["keys"].tolist() and c.tolist() == w["count"].tolist()
                    and sm.tolist() == w["sums"].tolist()):
                bad.append((name, i, q.shape, q.fact_first, q.n_fact, q.dim_first, q.n_dim, int(c.sum()),
                            int(w["count"].sum())))
    for b in bad:
        say("mismatch", b)
    for i in range(len(reqs)):
        q = R[i]
        assert alone[0][i].status == 0 and mixed[0][i].status == 0, i
        a = packed(setup, q, *alone, i)
        m = packed(setup, q, *mixed, i)
        w = expected(setup, q)
        for x, y in zip(a, m):
            assert x.tolist() == y.tolist(), (i, q.shape)
        assert a[0].tolist() == w["keys"].tolist(), (i, q.shape)
        assert a[1].tolist() == w["count"].tolist(), (i, q.shape)
        assert a[2].tolist() == w["sums"].tolist(), (i, q.shape)


def test_budget_admission_and_oversized_request(setup):
    reqs = wl.serving_requests(12, qps=5000.0, fact_lo=4.0, fact_hi=5.0, seed=wl.SERVE_SEED + 2)
    R = setup.requests(reqs)
    # room for about one join request at a time: admission serialises, nothing deadlocks
    budget = tq.Budget(24 << 20)
    arena = torch.empty(24 << 20, dtype=torch.uint8, device="cuda")
    res, keys, count, sums = tq.serve_run(setup.T, R, 4, budget, arena, 25)
    ok = [res[i].status for i in range(len(reqs))]
    assert all(s in (0, tq.TQ_ENOMEM) for s in ok)
    for i in range(len(reqs)):
        if res[i].status == 0:
            w = expected(setup, R[i])
            assert packed(setup, R[i], res, keys, count, sums, i)[1].tolist() == w["count"].tolist()
    assert budget.used == 0


def _join_requests(setup, n, seed):
    """Join requests only (shapes 1 and 2), all arriving at once."""
    reqs = [r for r in wl.serving_requests(4 * n, qps=1e9, fact_lo=4.5, fact_hi=5.3, seed=seed) if r.shape != 0][:n]
    return setup.requests(reqs)


def _equal_oracle(setup, R, run, i):
    k, c, sm = packed(setup, R[i], *run, i)
    w = expected(setup, R[i])
    return k.tolist() == w["keys"].tolist() and c.tolist() == w["count"].tolist() and sm.tolist() == w["sums"].tolist()


def test_history_reservations_are_smaller_and_results_unchanged(setup):
    """With the memory-use history, join requests after the first ones reserve
    tables for the kept fraction seen so far instead of the whole window, so
    more of them fit a tight budget at once; every result still equals the
    oracle, and uniform data never needs a retry."""
    R = _join_requests(setup, 24, wl.SERVE_SEED + 3)
    n = len(R)
    arena = torch.empty(24 << 20, dtype=torch.uint8, device="cuda")
    runs = {}
    for est in (0, 1):
        setup.T.estimate = est
        budget = tq.Budget(24 << 20)
        runs[est] = tq.serve_run(setup.T, R, 4, budget, arena, 25)
        assert budget.used == 0
    setup.T.estimate = 1
    on, off = runs[1][0], runs[0][0]
    for i in range(n):
        assert on[i].status == 0 and off[i].status == 0, i
        assert _equal_oracle(setup, R, runs[1], i), i
        assert _equal_oracle(setup, R, runs[0], i), i
        assert on[i].retries == 0 and off[i].retries == 0
        assert on[i].reserved_bytes <= off[i].reserved_bytes
    total_on = sum(on[i].reserved_bytes for i in range(n))
    total_off = sum(off[i].reserved_bytes for i in range(n))
    say(f"reserved: history {total_on / 2**20:.1f} MiB, whole windows {total_off / 2**20:.1f} MiB")
    assert total_on < total_off
    # only the requests admitted before any join had completed reserve for the whole window
    assert sum(on[i].reserved_bytes < off[i].reserved_bytes for i in range(n)) >= n // 2


@pytest.fixture(scope="module")
def sorted_setup():
    pool = tq.PagePool(1 << 20, 100, pinned=True)
    s = pipeline.ServingSetup(n0=4096, n_dim=120_000, n1=100_000, n2=65_536, batch_rows=16_384, pool=pool,
                              dim_sorted_by="date")
    yield s
    s.host.free()
    pool.close()


def test_retry_after_a_table_sized_too_small(sorted_setup):
    """Dimension sorted by date: windows at the start keep no row, so the
    history says nothing is kept; a later window inside the date range keeps
    every row, its table proves too small, and it runs again for the exact
    count recorded by the failed build."""
    s = sorted_setup
    kept = (s.dim["date"] >= 730) & (s.dim["date"] <= 1094)
    first_kept = int(np.argmax(kept))
    assert not kept[:16_000].any()
    R = (tq.Request * 5)()
    for i in range(5):
        q = R[i]
        q.shape, q.arrival_s, q.fact_first, q.n_fact = 1, 0.0, 16 * i, 50_000
        q.dim_first, q.n_dim = (0, 16_000) if i < 4 else ((first_kept + 15) // 16 * 16, 12_000)
    assert kept[R[4].dim_first:R[4].dim_first + 12_000].all()
    for est in (1, 0):
        s.T.estimate = est
        budget = tq.Budget(64 << 20)
        arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        run = tq.serve_run(s.T, R, 1, budget, arena, 25)
        res = run[0]
        say([(res[i].status, res[i].retries, res[i].reserved_bytes) for i in range(5)])
        assert budget.used == 0
        for i in range(5):
            assert res[i].status == 0, i
            assert _equal_oracle(s, R, run, i), i
        assert [res[i].retries for i in range(5)] == ([0, 0, 0, 0, 1] if est else [0] * 5)
        if est:
            assert res[1].reserved_bytes < res[0].reserved_bytes  # the history shrank the table
    s.T.estimate = 1
