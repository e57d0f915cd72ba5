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
from paper_2508_05029_amd.datagen import workloads as wl
from paper_2508_05029_amd.datagen.workloads import (FILTER_GROUPBY_QUERY, JOIN_AGG_QUERY, Factor, FilterGroupByQuery,
                                                     GroupKey, Pred, filter_groupby_tables, join_agg_tables)
from tests import brute
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


# ---------------------------------------------------------------- NULLs

def _with_nulls(n, density, seed, lo=-50, hi=50):
    """A column as (numpy int64 values, Arrow bitmap, Python list with None)."""
    rng = np.random.default_rng(seed)
    vals = rng.integers(lo, hi + 1, n).astype(np.int64)
    present = rng.random(n) >= density
    bits = np.packbits(present.astype(np.uint8), bitorder="little")
    return vals, bits, [int(v) if p else None for v, p in zip(vals, present)]


def _oracle_groups_nulls(got):
    out = []
    for g in range(len(got["count"])):
        key = None if got["key_null"][g] else int(got["keys"][g])
        sums = [int(s) if c else None for s, c in zip(got["sums"][g], got["nonnull"][g])]
        out.append((key, int(got["count"][g]), sums, [int(c) for c in got["nonnull"][g]]))
    return out


@pytest.mark.parametrize("seed,density", [(1, 0.0), (2, 0.1), (3, 0.5), (4, 0.9), (5, 1.0)])
def test_nullable_filter_groupby_matches_brute(seed, density):
    n = 90
    k, kb, kl = _with_nulls(n, density, seed * 10 + 1, 0, 6)
    v, vb, vl = _with_nulls(n, density, seed * 10 + 2, -(2 ** 62), 2 ** 62)
    w, wb, wl = _with_nulls(n, density, seed * 10 + 3, 0, 10)
    t = {"k": k, "v": v, "w": w}
    valid = {"k": kb, "v": vb, "w": wb}
    sums = [(Factor("v"),), (Factor("v"), Factor("w", -1, 10)), (Factor(None, 0, 7),)]
    q = FilterGroupByQuery(preds=[Pred("w", 2, 8)], key=GroupKey(("k",), 1, 7), sums=sums, avg_of=[])
    got = oracle.filter_groupby_nullable(t, valid, q)
    want = brute.brute_groupby_nulls({"k": kl, "v": vl, "w": wl}, [("w", 2, 8)], "k",
                                     [[(f.col, f.sign, f.add) for f in e] for e in sums], n)
    assert _oracle_groups_nulls(got) == [(key, c, s, cn) for key, c, s, cn, _ in want]
    for g, (_, _, _, cn, avgs) in enumerate(want):
        for j, a in enumerate(avgs):
            if a is not None:
                assert abs(got["avg"][g, j] - float(a)) <= 1e-12 * abs(float(a))


def test_nullable_without_nulls_equals_the_plain_oracle():
    t = wl.filter_groupby_tables(20_000, seed=77)
    q = wl.FILTER_GROUPBY_QUERY
    q1 = FilterGroupByQuery(preds=q.preds, key=GroupKey(("flagA",), 1, 3), sums=q.sums, avg_of=[])
    plain = oracle.filter_groupby(t, q1)
    n = 20_000
    ones = np.packbits(np.ones(n, np.uint8), bitorder="little")
    for valid in (None, {}, {c: ones for c in t}):
        got = oracle.filter_groupby_nullable(t, valid, q1)
        assert not got["key_null"].any()
        assert got["keys"].tolist() == plain["keys"][:, 0].tolist()
        assert got["count"].tolist() == plain["count"].tolist()
        assert got["sums"].tolist() == plain["sums"].tolist()
        assert (got["nonnull"] == got["count"][:, None]).all()
        assert got["avg"].tolist() == plain["avg"].tolist()
    dim, fact = wl.join_agg_tables(3_000, 12_000, seed=78)
    jq = JOIN_AGG_QUERY
    plain = oracle.join_agg(dim, fact, jq)
    got = oracle.join_agg_nullable(dim, None, fact, None, jq)
    assert got["join_rows"] == plain["join_rows"]
    assert got["keys"].tolist() == plain["keys"][:, 0].tolist()
    assert got["count"].tolist() == plain["count"].tolist() and got["sums"].tolist() == plain["sums"].tolist()


def test_nullable_all_null_values_and_keys():
    n = 40
    t = {"k": np.arange(n, dtype=np.int64) % 3, "v": np.arange(n, dtype=np.int64)}
    none = np.zeros((n + 7) // 8, np.uint8)
    q = FilterGroupByQuery(preds=[], key=GroupKey(("k",), 1, 3), sums=[(Factor("v"),)], avg_of=[])
    got = oracle.filter_groupby_nullable(t, {"v": none}, q)
    assert got["count"].tolist() == [14, 13, 13] and got["nonnull"][:, 0].tolist() == [0, 0, 0]
    assert got["sums"][:, 0].tolist() == [0, 0, 0]
    got = oracle.filter_groupby_nullable(t, {"k": none}, q)  # every key NULL: one group, listed as NULL
    assert got["key_null"].tolist() == [True] and got["count"].tolist() == [n]
    assert got["sums"][:, 0].tolist() == [n * (n - 1) // 2]


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_nullable_join_agg_matches_brute(seed):
    nd, nf = 30, 70
    key, kb, kl = _with_nulls(nd, 0.2, seed, 0, 15)
    grp, gb, gl = _with_nulls(nd, 0.2, seed + 100, 0, 3)
    date, db, dl = _with_nulls(nd, 0.1, seed + 200, 700, 1200)
    fk, fb, fl = _with_nulls(nf, 0.2, seed + 300, 0, 18)
    price, pb, plist = _with_nulls(nf, 0.2, seed + 400, 90_000, 10_500_000)
    disc, cb, cl = _with_nulls(nf, 0.2, seed + 500, 0, 10)
    dim = {"key": key, "group": grp.astype(np.int32), "date": date.astype(np.int32)}
    fact = {"fk": fk, "price": price, "disc": disc}
    q = JOIN_AGG_QUERY
    got = oracle.join_agg_nullable(dim, {"key": kb, "group": gb, "date": db}, fact,
                                   {"fk": fb, "price": pb, "disc": cb}, q)
    bpass = brute.brute_filter_nulls({"date": dl}, [(p.col, p.lo, p.hi) for p in q.build_preds], nd)
    pairs = brute.brute_join_nulls(kl, fl, bpass)
    assert got["join_rows"] == len(pairs)
    # group by the build payload over the pairs, by brute force
    rows = {"g": [gl[b] for _, b in pairs], "price": [plist[p] for p, _ in pairs], "disc": [cl[p] for p, _ in pairs]}
    exprs = [[(f.col, f.sign, f.add) for f in e] for e in q.sums]
    want = brute.brute_groupby_nulls(rows, [], "g", exprs, len(pairs))
    assert _oracle_groups_nulls(got) == [(k_, c, s, cn) for k_, c, s, cn, _ in want]


def test_golden_nulls():
    fx = _load("nulls_small.json")

    def col(values, dtype):
        present = np.array([x is not None for x in values], np.uint8)
        vals = np.array([0 if x is None else x for x in values], dtype=dtype)
        return vals, np.packbits(present, bitorder="little")

    g = fx["groupby"]
    t, valid = {}, {}
    for name, values in g["columns"].items():
        t[name], valid[name] = col(values, np.int64)
    sums = [tuple(Factor(*f) for f in e) for e in g["sums"]]
    q = FilterGroupByQuery(preds=[Pred(*p) for p in g["preds"]], key=GroupKey((g["key"],), 1, 10), sums=sums,
                           avg_of=[])
    got = oracle.filter_groupby_nullable(t, valid, q)
    e = g["expect"]
    assert [None if nl else int(k) for k, nl in zip(got["keys"], got["key_null"])] == e["keys"]
    assert got["count"].tolist() == e["count"]
    assert got["nonnull"].tolist() == e["nonnull"]
    assert [[int(s) if c else None for s, c in zip(r, cr)] for r, cr in zip(got["sums"], got["nonnull"])] == e["sums"]
    j = fx["join"]
    b, bv, p, pv = {}, {}, {}, {}
    for name, values in j["build"].items():
        b[name], bv[name] = col(values, np.int32 if name == "group" else np.int64)
    b["date"], bv["date"] = col([800] * len(j["build"]["key"]), np.int32)
    for name, values in j["probe"].items():
        p[name], pv[name] = col(values, np.int64)
    p["disc"], pv["disc"] = col([0] * len(j["probe"]["fk"]), np.int64)
    q = JOIN_AGG_QUERY  # window [730, 1094] passes every build row here; SUM(price * (100 - 0)) / 100
    got = oracle.join_agg_nullable(b, bv, p, pv, q)
    e = j["expect"]
    assert got["join_rows"] == e["join_rows"]
    assert [None if nl else int(k) for k, nl in zip(got["keys"], got["key_null"])] == e["keys"]
    assert got["count"].tolist() == e["count"]
    assert [int(s) // 100 for s in got["sums"][:, 0]] == e["sums"]
    assert got["nonnull"][:, 0].tolist() == e["nonnull"]


# ---------------------------------------------------------------------------
# dictionary-encoded strings

def _arrow(strings):
    off = np.zeros(len(strings) + 1, np.int32)
    off[1:] = np.cumsum([len(s) for s in strings])
    data = np.frombuffer(b"".join(strings), np.uint8).copy() if strings else np.zeros(0, np.uint8)
    return off, data


def _tricky_strings(n, seed):
    """Distinct byte strings that stress an equality test: the empty string,
    prefixes of one another, equal lengths that differ in one byte (first,
    middle, last), bytes 0x00 and >= 0x80."""
    rng = np.random.default_rng(seed)
    out = {b"", b"a", b"ab", b"abc", b"abd", b"bbc", b"\x00", b"\x00\x00", b"\xff", b"\x80a"}
    while len(out) < n:
        L = int(rng.integers(0, 12))
        out.add(bytes(rng.integers(0, 256, L).astype(np.uint8)) if rng.random() < 0.5
                else bytes(rng.choice(list(b"ab\x00\xff"), L).astype(np.uint8)))
    return sorted(out)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dict_unify_matches_a_python_dict(seed):
    pool = _tricky_strings(300, seed)
    rng = np.random.default_rng(seed)
    build = [pool[i] for i in rng.permutation(len(pool))[:200]]
    probe = [pool[i] for i in rng.permutation(len(pool))[:250]]
    where = {s: j for j, s in enumerate(build)}
    want = [where.get(s, -1) for s in probe]
    got = oracle.dict_unify(_arrow(build), _arrow(probe))
    assert got.tolist() == want
    assert (got == -1).sum() == len(set(probe) - set(build)) > 0


def test_dict_unify_empty_sides():
    assert oracle.dict_unify(_arrow([]), _arrow([b"x", b""])).tolist() == [-1, -1]
    assert oracle.dict_unify(_arrow([b"x", b""]), _arrow([])).tolist() == []
    assert oracle.dict_unify(_arrow([b"x", b""]), _arrow([b"", b"x", b"y"])).tolist() == [1, 0, -1]


def test_string_workload_dictionaries_are_distinct_and_overlap_by_three_quarters():
    T = wl.string_join_tables(4000, 100)
    b = oracle.decode(T.build_dict, np.arange(4000))
    p = oracle.decode(T.probe_dict, np.arange(4000))
    assert len(set(b)) == 4000 and len(set(p)) == 4000
    assert len(set(b) & set(p)) == 3000
    # the id after the last '#' names the string
    assert all(int(s.rsplit(b"#", 1)[1]) < 4000 for s in b)


@pytest.mark.parametrize("seed", [21, 22])
def test_join_agg_strings_matches_brute(seed):
    """Nested loops over the decoded strings: a pair joins when its strings are
    equal and neither key is NULL."""
    nd, nf = 40, 90
    T = wl.string_join_tables(nd, nf, seed=seed)
    rng = np.random.default_rng(seed)
    kvalid = rng.random(nd) >= 0.15
    fvalid = rng.random(nf) >= 0.15
    dv = {"key": np.packbits(kvalid.astype(np.uint8), bitorder="little")}
    fv = {"fk": np.packbits(fvalid.astype(np.uint8), bitorder="little")}
    q = JOIN_AGG_QUERY
    got = oracle.join_agg_strings(T.build_dict, T.dim, dv, T.probe_dict, T.fact, fv, q)
    bs = oracle.decode(T.build_dict, T.dim["key"], dv["key"])
    ps = oracle.decode(T.probe_dict, T.fact["fk"], fv["fk"])
    groups = {}
    npairs = 0
    for p in range(nf):
        for b in range(nd):
            if bs[b] is None or ps[p] is None or bs[b] != ps[p]:
                continue
            if not (q.build_preds[0].lo <= T.dim["date"][b] <= q.build_preds[0].hi):
                continue
            npairs += 1
            g = int(T.dim["group"][b])
            c, s = groups.get(g, (0, [0] * len(q.sums)))
            vals = [brute_expr_exact(T.fact, [(f.col, f.sign, f.add) for f in e], p) for e in q.sums]
            groups[g] = (c + 1, [to_i64(a + v) for a, v in zip(s, vals)])
    assert got["join_rows"] == npairs > 0
    assert got["keys"].tolist() == sorted(groups)
    assert got["count"].tolist() == [groups[g][0] for g in sorted(groups)]
    assert got["sums"].tolist() == [groups[g][1] for g in sorted(groups)]


def test_first_occurrence_matches_nested_loops():
    rng = np.random.default_rng(7)
    pool = _tricky_strings(40, 8)
    strs = [pool[i] for i in rng.integers(0, len(pool), 300)]
    got = oracle.first_occurrence(_arrow(strs))
    want = [min(j for j in range(len(strs)) if strs[j] == strs[i]) for i in range(len(strs))]
    assert got.tolist() == want
    assert oracle.first_occurrence(_arrow([])).tolist() == []
