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


def packed(setup, q, res, keys, count, sums, avg, i):
    """(keys, COUNT, SUMs, AVGs) of request i in the oracle's layout."""
    g = res[i].ngroups
    nsum = 5 if q.shape == 0 else 1
    k = keys[i, :g]
    if q.shape == 0:  # the packed key flagA * 2 + flagB
        k = np.stack([k // 2, k % 2], axis=1)
    else:
        k = k.reshape(-1, 1)
    return k, count[i, :g], sums[i, :g, :nsum], avg[i, :g, :nsum]


def same_as_oracle(got, want):
    """Integers bit-exact; AVG within 1e-12 relative (both sides divide once in IEEE double)."""
    k, c, sm, av = got
    if not (k.tolist() == want["keys"].tolist() and c.tolist() == want["count"].tolist()
            and sm.tolist() == want["sums"].tolist()):
        return False
    return bool(np.all(np.abs(av - want["avg"]) <= 1e-12 * np.abs(want["avg"])))


def reservation(setup, q, rows=None):
    """The device bytes a request reserves, by the rule tq_serve_run documents
    (each piece rounded up to 256 bytes, at least 8), with the join table sized
    for the whole dimension window (no memory-use history)."""
    al = lambda b: (max(b, 8) + 255) // 256 * 256  # noqa: E731
    T = setup.T
    domain, nsum = (T.fg_domain, T.fg_nsum) if q.shape == 0 else (T.join_domain, T.join_nsum)
    table = 0 if q.shape == 0 else tq.join_table_bytes(q.n_dim if rows is None else rows, T.load_factor)
    staging = 0
    if q.shape == 2:
        pages = max(len(setup.host.batches[b][3]) for b in range(q.fact_first, q.fact_first + q.n_fact))
        staging = pages * setup.host.pool.page_bytes * T.nslots
    return sum(al(b) for b in (tq.groupby_state_bytes(domain, nsum), table, 8 * domain, 8 * domain,
                               8 * domain * nsum, 8 * domain * nsum, 8, staging, 64))


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
            got = packed(setup, q, *run, i)
            if not same_as_oracle(got, w):
                bad.append((name, i, q.shape, q.fact_first, q.n_fact, q.dim_first, q.n_dim, int(got[1].sum()),
                            int(w["count"].sum())))
    for b in bad:
        say("mismatch", b)
    for i in range(len(reqs)):
        q = R[i]
        assert alone[0][i].status == 0 and mixed[0][i].status == 0, i
        a = packed(setup, q, *alone, i)
        m = packed(setup, q, *mixed, i)
        # alone and in the mix: the same bits, AVG included (one division of the same integers)
        for x, y in zip(a, m):
            assert x.tolist() == y.tolist(), (i, q.shape)
        assert same_as_oracle(a, expected(setup, q)), (i, q.shape)
    assert not bad


def test_budget_admission_and_oversized_request(setup):
    """A budget with room for about one join request at a time: admission
    serialises and nothing deadlocks; exactly the join requests whose documented
    reservation exceeds the cap run split into hash partitions (one after
    another, each table within the cap), and every result, split or not, equals
    the oracle."""
    reqs = wl.serving_requests(12, qps=5000.0, fact_lo=4.0, fact_hi=5.0, seed=wl.SERVE_SEED + 2)
    base = setup.requests(reqs)
    rows = [(base[i].shape, base[i].fact_first, base[i].n_fact, base[i].dim_first, base[i].n_dim, base[i].arrival_s)
            for i in range(len(reqs))]
    # two requests that do not fit whole: joins over the whole dimension (a 2^18-slot table, 9.7 MB), one
    # in the middle of the queue and one at its end; they must run split without holding up the others
    rows.insert(4, (1, 0, 50_000, 0, setup.n_dim, rows[3][5]))
    rows.append((2, 0, 2, 0, setup.n_dim, rows[-1][5]))
    R = (tq.Request * len(rows))()
    for i, (shape, ff, nf, df, nd, at) in enumerate(rows):
        R[i].shape, R[i].fact_first, R[i].n_fact, R[i].dim_first, R[i].n_dim, R[i].arrival_s = shape, ff, nf, df, nd, at
    reqs = rows
    setup.T.estimate = 0  # tables for whole windows, so each reservation is known in advance
    cap = 8 << 20
    try:
        budget = tq.Budget(cap)
        arena = torch.empty(cap, dtype=torch.uint8, device="cuda")
        run = tq.serve_run(setup.T, R, 4, budget, arena, 25)
    finally:
        setup.T.estimate = 1
    res = run[0]
    need = [reservation(setup, R[i]) for i in range(len(reqs))]
    say(f"reservations (MiB): {[round(b / 2**20, 1) for b in need]}, cap {cap / 2**20:.0f}")
    assert [i for i in range(len(reqs)) if need[i] > cap] == [4, len(reqs) - 1]
    for i in range(len(reqs)):
        assert res[i].status == 0, i
        if need[i] > cap:
            say(f"request {i}: split into {res[i].splits} partitions, reserved {res[i].reserved_bytes / 2**20:.1f} MiB")
            assert res[i].splits > 1 and res[i].reserved_bytes <= cap, i
        else:
            assert res[i].splits == 1, i
            assert res[i].reserved_bytes == need[i], i
        assert same_as_oracle(packed(setup, R[i], *run, i), expected(setup, R[i])), i
    assert budget.used == 0


def test_requests_that_cannot_fit_even_split_fail_alone(setup):
    """A budget that holds a filter + group-by request but no join request, not
    even split 256 ways (its group-by state alone is larger): the joins complete
    at once with TQ_ENOMEM, the others run and equal the oracle, nothing waits
    forever."""
    reqs = wl.serving_requests(12, qps=5000.0, fact_lo=4.0, fact_hi=5.0, seed=wl.SERVE_SEED + 5)
    R = setup.requests(reqs)
    setup.T.estimate = 0
    cap = 400 << 10
    try:
        budget = tq.Budget(cap)
        arena = torch.empty(cap, dtype=torch.uint8, device="cuda")
        run = tq.serve_run(setup.T, R, 3, budget, arena, 25)
    finally:
        setup.T.estimate = 1
    res = run[0]
    shapes = [R[i].shape for i in range(len(reqs))]
    assert 0 in shapes and any(x != 0 for x in shapes)
    for i in range(len(reqs)):
        if R[i].shape == 0:
            assert res[i].status == 0, i
            assert reservation(setup, R[i]) <= cap
            assert same_as_oracle(packed(setup, R[i], *run, i), expected(setup, R[i])), i
        else:
            assert res[i].status == tq.TQ_ENOMEM, i
    assert budget.used == 0


def test_split_join_equals_whole_join(setup):
    """The same join requests served whole (a large budget) and split into hash
    partitions (a budget below each one's whole reservation): equal results,
    equal to the oracle."""
    # device-resident joins only (a streamed one reserves its staging slots whole, which no
    # split makes smaller)
    reqs = [r for r in wl.serving_requests(40, qps=1e9, fact_lo=4.5, fact_hi=5.3, seed=wl.SERVE_SEED + 6)
            if r.shape == 1][:6]
    R = setup.requests(reqs)
    n = len(R)
    setup.T.estimate = 0
    try:
        big = tq.Budget(256 << 20)
        arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        whole = tq.serve_run(setup.T, R, 2, big, arena, 25)
        cap = min(reservation(setup, R[i]) for i in range(n)) - 1
        small = tq.Budget(cap)
        split = tq.serve_run(setup.T, R, 2, small, arena, 25)
    finally:
        setup.T.estimate = 1
    for i in range(n):
        assert whole[0][i].status == 0 and split[0][i].status == 0, i
        assert whole[0][i].splits == 1 and split[0][i].splits > 1, i
        a = packed(setup, R[i], *whole, i)
        b = packed(setup, R[i], *split, i)
        for x, y in zip(a, b):
            assert x.tolist() == y.tolist(), i
        assert same_as_oracle(b, expected(setup, R[i])), i


def _join_requests(setup, n, seed):
    """Join requests only (shapes 1 and 2), all arriving at once."""
    reqs = [r for r in wl.serving_requests(4 * n, qps=1e9, fact_lo=4.5, fact_hi=5.3, seed=seed) if r.shape != 0][:n]
    return setup.requests(reqs)


def _equal_oracle(setup, R, run, i):
    return same_as_oracle(packed(setup, R[i], *run, i), expected(setup, R[i]))


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
