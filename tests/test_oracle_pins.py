"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each group pins one step of the path to something independent: nested-loop
brute force with Python integers, closed forms, a special case that reduces to
a numpy routine, invariants (join cardinality, partition conservation), exact
rationals for AVG, and hand-worked fixtures under tests/golden/.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2508_05029_amd.datagen import uniform, permutation
from paper_2508_05029_amd.datagen.workloads import (FILTER_GROUPBY_QUERY, JOIN_AGG_QUERY, Factor, Pred,
                                                     filter_groupby_tables, join_agg_tables)
from tests.brute import (brute_expr_exact, brute_filter, brute_groupby, brute_join, brute_partition_id,
                         to_i64)

I64_MIN, I64_MAX = -(2 ** 63), 2 ** 63 - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_table(n, seed):
    rng = np.random.default_rng(seed)
    return {
        "a": rng.integers(-5, 6, n).astype(np.int64),
        "b": rng.integers(0, 4, n).astype(np.int32),
        "c": rng.integers(0, 256, n).astype(np.uint8),
        "v": rng.integers(-10**12, 10**12, n).astype(np.int64),
        "w": rng.integers(-3, 4, n).astype(np.int64),
    }


def as_tuples(preds):
    return [(p.col, p.lo, p.hi) for p in preds]


def as_expr(e):
    return [(f.col, f.sign, f.add) for f in e]


# ---------------------------------------------------------------- selection

@pytest.mark.parametrize("seed", range(6))
def test_filter_matches_brute(seed):
    t = tiny_table(200, seed)
    preds = [Pred("a", -2, 3), Pred("c", 10, 200), Pred("b", 1, 1)][: 1 + seed % 3]
    m = oracle.filter_mask(t, preds)
    assert list(m.astype(bool)) == brute_filter(t, as_tuples(preds), 200)


def test_filter_widening_of_unsigned_and_extremes():
    t = {"c": np.array([0, 127, 128, 255], dtype=np.uint8),
         "i": np.array([I64_MIN, -1, 0, I64_MAX], dtype=np.int64),
         "s": np.array([-2**31, -1, 0, 2**31 - 1], dtype=np.int32)}
    assert list(oracle.filter_mask(t, [Pred("c", 128, 255)])) == [0, 0, 1, 1]   # zero extension
    assert list(oracle.filter_mask(t, [Pred("s", I64_MIN, -1)])) == [1, 1, 0, 0]  # sign extension
    assert list(oracle.filter_mask(t, [Pred("i", I64_MIN, I64_MAX)])) == [1, 1, 1, 1]
    assert list(oracle.filter_mask(t, [Pred("i", 1, 0)])) == [0, 0, 0, 0]  # empty range


@pytest.mark.parametrize("D,c", [(2526, 2436), (7, 3), (100, 0), (100, 99)])
def test_filter_closed_form_count(D, c):
    n = 100_003
    t = {"date": (np.arange(n) % D).astype(np.int32)}
    m = oracle.filter_mask(t, [Pred("date", I64_MIN, c)])
    full, rem = divmod(n, D)
    expect = full * (c + 1) + min(rem, c + 1)
    assert int(m.sum()) == expect


# ---------------------------------------------------------------- projection

@pytest.mark.parametrize("seed", range(4))
def test_project_matches_brute(seed):
    t = tiny_table(150, seed)
    expr = (Factor("v", 1, 0), Factor("w", -1, 100), Factor("b", 1, 7))
    out, ovf = oracle.project(t, expr)
    for r in range(150):
        exact = brute_expr_exact(t, as_expr(expr), r)
        assert out[r] == to_i64(exact)


def test_project_wraps_mod_2_64_and_flags_overflow():
    t = {"x": np.array([I64_MAX, I64_MIN, 2**62, -(2**62), 3], dtype=np.int64)}
    out, ovf = oracle.project(t, (Factor("x", 1, 0), Factor(None, 1, 2)))
    assert list(out) == [to_i64(I64_MAX * 2), to_i64(I64_MIN * 2), to_i64(2**63), to_i64(-(2**63)), 6]
    assert list(ovf) == [1, 1, 1, 0, 0]
    out, ovf = oracle.project(t, (Factor("x", -1, 0),))  # -INT64_MIN wraps to itself
    assert out[1] == I64_MIN and ovf[1] == 1 and ovf[0] == 0


def test_project_closed_form_zero_discount_and_tax():
    n = 10_000
    p = uniform(n, 90_000, 10_500_000, np.int64, 1, 1)
    t = {"price": p, "disc": np.zeros(n, np.int64), "tax": np.zeros(n, np.int64)}
    e = FILTER_GROUPBY_QUERY.sums[3]
    out, _ = oracle.project(t, e)
    assert int(out.sum()) == 10_000 * int(p.sum())


# ---------------------------------------------------------------- group-by

@pytest.mark.parametrize("seed", range(6))
def test_groupby_matches_brute(seed):
    t = tiny_table(250, seed)
    preds = [Pred("a", -3, 4)] if seed % 2 else []
    keys = ["b", "c"] if seed % 3 == 0 else ["a"]
    exprs = [(Factor("v", 1, 0),), (Factor("v", 1, 0), Factor("w", -1, 100)), (Factor("w", 1, 0),)]
    mask = oracle.filter_mask(t, preds) if preds else None
    vals = [oracle.project(t, e)[0] for e in exprs]
    got = oracle.groupby([t[k] for k in keys], vals, mask)
    want = brute_groupby(t, as_tuples(preds), keys, [as_expr(e) for e in exprs], 250)
    assert len(got["count"]) == len(want)
    for g, (k, cnt, sums, avgs, _) in enumerate(want):
        assert tuple(got["keys"][g]) == k
        assert got["count"][g] == cnt
        assert list(got["sums"][g]) == sums
        for j, a in enumerate(avgs):
            assert got["avg"][g][j] == float(a)  # one IEEE RNE rounding of the exact ratio


def test_groupby_closed_form_arithmetic_series():
    n, G = 1_000_000, 7
    r = np.arange(n, dtype=np.int64)
    got = oracle.groupby([r % G], [r])
    for g in range(G):
        m = (n - 1 - g) // G + 1  # number of rows r = g + G i < n
        assert got["count"][g] == m
        assert got["sums"][g][0] == m * g + G * m * (m - 1) // 2


def test_groupby_empty_and_all_filtered():
    k = np.array([1, 2, 3], dtype=np.int64)
    got = oracle.groupby([k], [k], np.zeros(3, np.uint8))
    assert len(got["count"]) == 0
    got = oracle.groupby([np.zeros(0, np.int64)], [np.zeros(0, np.int64)])
    assert len(got["count"]) == 0


def test_groupby_sum_wraps_and_is_flagged():
    k = np.zeros(3, np.int64)
    v = np.array([I64_MAX, 1, 1], dtype=np.int64)
    got = oracle.groupby([k], [v])
    assert got["sums"][0][0] == to_i64(I64_MAX + 2) and got["overflow"][0][0] == 1


def test_filter_groupby_config_against_numpy_add_at():
    """Full 1M-row filter+group-by: np.add.at (exact int64) and np.bincount."""
    t = filter_groupby_tables()
    q = FILTER_GROUPBY_QUERY
    got = oracle.filter_groupby(t, q)
    m = t["date"] <= 2436
    g = (t["flagA"].astype(np.int64) * 2 + t["flagB"])[m]
    p, d, tx = t["price"][m], t["disc"][m], t["tax"][m]
    cols = [t["qty"][m], p, p * (100 - d), p * (100 - d) * (100 + tx), d]
    cnt = np.bincount(g, minlength=6)
    assert list(got["count"]) == list(cnt[cnt > 0])
    assert [tuple(k) for k in got["keys"]] == [(a, b) for a in range(3) for b in range(2)]
    for j, c in enumerate(cols):
        s = np.zeros(6, np.int64)
        np.add.at(s, g, c)
        assert list(got["sums"][:, j]) == list(s)
    assert not got["overflow"].any()
    # AVG within 1e-12 of the exact rational
    for gi in range(6):
        for j in q.avg_of:
            exact = Fraction(int(got["sums"][gi][j]), int(got["count"][gi]))
            assert abs(Fraction(float(got["avg"][gi][j])) - exact) <= Fraction(1, 10**12) * abs(exact)
    assert int(got["count"].sum()) == int(m.sum())


# ---------------------------------------------------------------- join

def _join_cases():
    rng = np.random.default_rng(5)
    yield rng.integers(0, 30, 80), rng.integers(0, 40, 120)                       # dups on both sides
    yield np.array([I64_MAX, I64_MIN + 1, -1, 0, 5]), np.array([5, -1, I64_MAX, 7, I64_MIN + 1, 5])
    yield np.zeros(0, np.int64), np.arange(10)                                    # empty build
    yield np.arange(10), np.zeros(0, np.int64)                                    # empty probe
    yield np.arange(0, 2**20, 2**16) * 3, np.arange(0, 2**20, 2**16) * 3          # same-slot collisions


@pytest.mark.parametrize("case", range(5))
def test_join_matches_brute(case):
    bk, pk = list(_join_cases())[case]
    bk = np.asarray(bk, np.int64)
    pk = np.asarray(pk, np.int64)
    total, pr, br = oracle.join_pairs(bk, pk)
    want = brute_join(bk, pk)
    assert total == len(want)
    assert list(zip(pr.tolist(), br.tolist())) == want


def test_join_with_masks_matches_brute():
    rng = np.random.default_rng(9)
    bk, pk = rng.integers(0, 20, 60), rng.integers(0, 20, 90)
    bm, pm = rng.integers(0, 2, 60).astype(np.uint8), rng.integers(0, 2, 90).astype(np.uint8)
    total, pr, br = oracle.join_pairs(bk, pk, bm, pm)
    assert list(zip(pr.tolist(), br.tolist())) == brute_join(bk, pk, bm, pm)


def test_join_cardinality_invariant():
    rng = np.random.default_rng(11)
    bk, pk = rng.integers(0, 5000, 20000), rng.integers(0, 7000, 50000)
    total, _, _ = oracle.join_pairs(bk, pk, with_pairs=False)
    ub, cb = np.unique(bk, return_counts=True)
    up, cp = np.unique(pk, return_counts=True)
    common, ib, ip = np.intersect1d(ub, up, return_indices=True)
    assert total == int((cb[ib] * cp[ip]).sum())


def test_join_agg_config_against_permutation_gather():
    """Dimension keys are a permutation of 0..N-1, so the join is a gather."""
    dim, fact = join_agg_tables()
    q = JOIN_AGG_QUERY
    got = oracle.join_agg(dim, fact, q)
    inv = np.empty(len(dim["key"]), np.int64)
    inv[dim["key"]] = np.arange(len(dim["key"]))
    row = inv[fact["fk"]]
    ok = (dim["date"][row] >= 730) & (dim["date"][row] <= 1094)
    grp = dim["group"][row][ok].astype(np.int64)
    val = (fact["price"] * (100 - fact["disc"]))[ok]
    cnt = np.bincount(grp, minlength=25)
    s = np.zeros(25, np.int64)
    np.add.at(s, grp, val)
    assert got["join_rows"] == int(ok.sum())
    assert list(got["keys"][:, 0]) == [g for g in range(25) if cnt[g] > 0]
    assert list(got["count"]) == list(cnt[cnt > 0])
    assert list(got["sums"][:, 0]) == list(s[cnt > 0])


# ---------------------------------------------------------------- partition

@pytest.mark.parametrize("bits", [0, 1, 3, 8])
def test_partition_matches_brute_and_is_stable(bits):
    rng = np.random.default_rng(bits)
    keys = np.concatenate([rng.integers(-10**15, 10**15, 300), [I64_MIN, I64_MAX, 0, -1]]).astype(np.int64)
    perm, offs = oracle.partition(keys, bits)
    pid = [brute_partition_id(k, bits) for k in keys]
    expect = sorted(range(len(keys)), key=lambda r: (pid[r], r))
    assert list(perm) == expect
    for p in range(1 << bits):
        assert offs[p + 1] - offs[p] == pid.count(p)


def test_partition_conservation_and_membership():
    keys = permutation(100_000, 3, 0)
    vals = uniform(100_000, -10**15, 10**15, np.int64, 3, 1)
    perm, offs = oracle.partition(keys, 8)
    assert offs[0] == 0 and offs[-1] == len(keys)
    pid = oracle.partition_ids(keys, 8)
    assert sorted(perm.tolist()) == list(range(len(keys)))
    for p in range(256):
        rows = perm[offs[p]:offs[p + 1]]
        assert (pid[rows] == p).all()
    assert int(vals[perm].sum()) == int(vals.sum())


def test_partition_hash_is_the_fibonacci_multiplier():
    # k = 1 gives the multiplier itself: top byte 0x9E = 158
    assert oracle.partition_ids(np.array([1], np.int64), 8)[0] == 0x9E
    assert oracle.partition_ids(np.array([0], np.int64), 8)[0] == 0


# ---------------------------------------------------------------- hand-worked fixtures

def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_golden_filter_groupby():
    fx = _load("filter_groupby_small.json")
    t = {k: np.array(v, dtype=fx["dtypes"][k]) for k, v in fx["columns"].items()}
    preds = [Pred(*p) for p in fx["preds"]]
    vals = [oracle.project(t, [Factor(*f) for f in e])[0] for e in fx["sums"]]
    got = oracle.groupby([t[k] for k in fx["keys"]], vals, oracle.filter_mask(t, preds))
    assert got["keys"].tolist() == fx["expect"]["keys"]
    assert got["count"].tolist() == fx["expect"]["count"]
    assert got["sums"].tolist() == fx["expect"]["sums"]


def test_golden_join_agg():
    fx = _load("join_agg_small.json")
    b = {k: np.array(v, dtype=fx["build_dtypes"][k]) for k, v in fx["build"].items()}
    p = {k: np.array(v, dtype=fx["probe_dtypes"][k]) for k, v in fx["probe"].items()}
    bm = oracle.filter_mask(b, [Pred(*x) for x in fx["build_preds"]])
    total, pr, br = oracle.join_pairs(b["key"], p["fk"], bm)
    assert total == fx["expect"]["join_rows"]
    assert [list(x) for x in zip(pr.tolist(), br.tolist())] == fx["expect"]["pairs"]
    q = JOIN_AGG_QUERY
    got = oracle.join_agg(b, p, q)
    assert got["keys"][:, 0].tolist() == fx["expect"]["keys"]
    assert got["count"].tolist() == fx["expect"]["count"]
    assert got["sums"].tolist() == fx["expect"]["sums"]


def test_golden_join_duplicate_keys():
    fx = _load("join_dup_keys.json")
    total, pr, br = oracle.join_pairs(np.array(fx["build_keys"]), np.array(fx["probe_keys"]))
    assert total == fx["expect"]["cardinality"]
    assert [list(x) for x in zip(pr.tolist(), br.tolist())] == fx["expect"]["pairs"]
