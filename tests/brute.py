"""Brute-force nested-loop evaluation with Python integers (tiny inputs only).

A third, independent statement of the relational definitions: lists and loops,
unbounded Python integers reduced modulo 2^64 only at the end, a linear search
for each group key, every build row against every probe row.
"""
from fractions import Fraction

M64 = 1 << 64
PHI = 0x9E3779B97F4A7C15


def to_i64(x: int) -> int:
    x %= M64
    return x - M64 if x >= (1 << 63) else x


def brute_filter(cols, preds, n):
    out = []
    for r in range(n):
        ok = True
        for (name, lo, hi) in preds:
            v = int(cols[name][r])
            if not (lo <= v <= hi):
                ok = False
        out.append(ok)
    return out


def brute_expr_exact(cols, expr, r):
    """Exact (unbounded) value of a product of affine factors at row r."""
    v = 1
    for (name, sign, add) in expr:
        x = 0 if name is None else int(cols[name][r])
        v *= sign * x + add
    return v


def brute_groupby(cols, preds, key_names, exprs, n):
    passing = brute_filter(cols, preds, n)
    keys, counts, sums = [], [], []
    for r in range(n):
        if not passing[r]:
            continue
        k = tuple(int(cols[c][r]) for c in key_names)
        idx = -1
        for i, kk in enumerate(keys):  # linear search, on purpose
            if kk == k:
                idx = i
                break
        if idx < 0:
            keys.append(k)
            counts.append(0)
            sums.append([0] * len(exprs))
            idx = len(keys) - 1
        counts[idx] += 1
        for j, e in enumerate(exprs):
            sums[idx][j] += brute_expr_exact(cols, e, r)
    order = sorted(range(len(keys)), key=lambda i: keys[i])
    return [(keys[i], counts[i], [to_i64(s) for s in sums[i]],
             [Fraction(to_i64(s), counts[i]) for s in sums[i]], sums[i]) for i in order]


def brute_join(bkeys, pkeys, bpass=None, ppass=None):
    pairs = []
    for p in range(len(pkeys)):
        if ppass is not None and not ppass[p]:
            continue
        for b in range(len(bkeys)):
            if bpass is not None and not bpass[b]:
                continue
            if int(bkeys[b]) == int(pkeys[p]):
                pairs.append((p, b))
    return pairs


def brute_partition_id(key: int, bits: int) -> int:
    if bits == 0:
        return 0
    return ((int(key) % M64) * PHI % M64) >> (64 - bits)


# ---------------------------------------------------------------- NULLs
# Columns here are Python lists whose NULL entries are None (no bitmaps), and
# SQL's rules are applied row by row: a predicate over None is not true, a
# product with a None factor is None, SUM/COUNT(e)/AVG skip None, COUNT(*) does
# not, None group keys form one group (sorted last), None join keys match
# nothing.

def brute_filter_nulls(cols, preds, n):
    out = []
    for r in range(n):
        ok = True
        for (name, lo, hi) in preds:
            v = cols[name][r]
            if v is None or not (lo <= int(v) <= hi):
                ok = False
        out.append(ok)
    return out


def brute_expr_nulls(cols, expr, r):
    v = 1
    for (name, sign, add) in expr:
        if name is None:
            x = 0
        else:
            x = cols[name][r]
            if x is None:
                return None
            x = int(x)
        v *= sign * x + add
    return v


def brute_groupby_nulls(cols, preds, key_name, exprs, n):
    """[(key or None, COUNT(*), [SUM_j or None], [COUNT_j], [AVG_j as Fraction or None])],
    non-NULL keys ascending, then the NULL key."""
    passing = brute_filter_nulls(cols, preds, n)
    groups = []  # [key, count, sums, counts]
    for r in range(n):
        if not passing[r]:
            continue
        k = cols[key_name][r]
        k = None if k is None else int(k)
        found = None
        for g in groups:  # linear search; None equals None here (SQL GROUP BY)
            if g[0] == k:
                found = g
                break
        if found is None:
            found = [k, 0, [0] * len(exprs), [0] * len(exprs)]
            groups.append(found)
        found[1] += 1
        for j, e in enumerate(exprs):
            v = brute_expr_nulls(cols, e, r)
            if v is not None:
                found[2][j] += v
                found[3][j] += 1
    groups.sort(key=lambda g: (g[0] is None, 0 if g[0] is None else g[0]))
    out = []
    for k, c, s, cn in groups:
        sums = [to_i64(x) if m else None for x, m in zip(s, cn)]
        avgs = [Fraction(to_i64(x), m) if m else None for x, m in zip(s, cn)]
        out.append((k, c, sums, cn, avgs))
    return out


def brute_join_nulls(bkeys, pkeys, bpass=None, ppass=None):
    pairs = []
    for p in range(len(pkeys)):
        if (ppass is not None and not ppass[p]) or pkeys[p] is None:
            continue
        for b in range(len(bkeys)):
            if (bpass is not None and not bpass[b]) or bkeys[b] is None:
                continue
            if int(bkeys[b]) == int(pkeys[p]):
                pairs.append((p, b))
    return pairs
