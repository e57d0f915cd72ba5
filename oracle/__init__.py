"""CPU oracle for the columnar query hot path (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package; the product path never does, and it shares no code with
the GPU library. The arithmetic lives in ``oracle.c`` (plain C, built into
``liboracle.so``); this wrapper only marshals numpy arrays.

What it computes is the plain relational definition of each step (the paper
delegates its operators to a GPU library and gives them no semantics of its
own, Section 2): selection, projection with int64 arithmetic modulo 2^64,
inner equi-join, group-by with COUNT/SUM/AVG, and the 64-bit multiplicative
hash partition of Section 3.2. Parity pins: see ``tests/test_oracle_pins.py``
(brute force, closed forms, library special cases, invariants).

Query descriptions are duck-typed: predicates have ``col, lo, hi``; factors
have ``col, sign, add``; expressions are sequences of factors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32)]


_vp, _i64, _i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        L.oc_filter.restype = _i64
        L.oc_filter.argtypes = [_vp, _i64, _i32, _vp, _vp, _vp, _vp]
        L.oc_project.restype = None
        L.oc_project.argtypes = [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp]
        L.oc_groupby.restype = _i64
        L.oc_groupby.argtypes = [_i64, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i64]
        L.oc_join.restype = _i64
        L.oc_join.argtypes = [_vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _i64]
        L.oc_partition_ids.restype = None
        L.oc_partition_ids.argtypes = [_vp, _i64, _i32, _vp]
        L.oc_partition.restype = None
        L.oc_partition.argtypes = [_vp, _i64, _i32, _vp, _vp]
        L.oc_filter_nullable.restype = _i64
        L.oc_filter_nullable.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp]
        L.oc_project_nullable.restype = None
        L.oc_project_nullable.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp]
        L.oc_groupby_nullable.restype = _i64
        L.oc_groupby_nullable.argtypes = [_i64, _vp, _Col, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64]
        L.oc_dict_unify.restype = None
        L.oc_dict_unify.argtypes = [_vp, _vp, _i64, _vp, _vp, _i64, _vp]
        _lib = L
    return _lib


_WIDTH = {np.dtype(np.uint8): 1, np.dtype(np.int32): 4, np.dtype(np.int64): 8}


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _cols(arrays: Sequence[np.ndarray]):
    arr = (_Col * max(1, len(arrays)))()
    for i, a in enumerate(arrays):
        assert a.flags["C_CONTIGUOUS"], "oracle columns must be contiguous"
        arr[i].data = a.ctypes.data
        arr[i].width = _WIDTH[a.dtype]
    return arr


def filter_mask(table: Dict[str, np.ndarray], preds) -> np.ndarray:
    """uint8 mask of the rows that satisfy every predicate (selection)."""
    n = len(next(iter(table.values())))
    names = sorted({p.col for p in preds})
    cols = [np.ascontiguousarray(table[c]) for c in names]
    pcol = np.array([names.index(p.col) for p in preds], dtype=np.int32)
    lo = np.array([p.lo for p in preds], dtype=np.int64)
    hi = np.array([p.hi for p in preds], dtype=np.int64)
    mask = np.empty(n, dtype=np.uint8)
    lib().oc_filter(_cols(cols), n, len(preds), _p(pcol), _p(lo), _p(hi), _p(mask))
    return mask


def project(table: Dict[str, np.ndarray], expr, n: Optional[int] = None):
    """Evaluate one product expression for every row. Returns (values, overflow)."""
    if n is None:
        n = len(next(iter(table.values())))
    names = sorted({f.col for f in expr if f.col is not None})
    cols = [np.ascontiguousarray(table[c]) for c in names]
    fcol = np.array([-1 if f.col is None else names.index(f.col) for f in expr], dtype=np.int32)
    fsign = np.array([f.sign for f in expr], dtype=np.int64)
    fadd = np.array([f.add for f in expr], dtype=np.int64)
    out = np.empty(n, dtype=np.int64)
    ovf = np.empty(n, dtype=np.uint8)
    lib().oc_project(_cols(cols), n, len(expr), _p(fcol), _p(fsign), _p(fadd), _p(out), _p(ovf))
    return out, ovf


def groupby(key_cols: Sequence[np.ndarray], values: Sequence[np.ndarray], mask: Optional[np.ndarray] = None,
            max_groups: Optional[int] = None) -> dict:
    """Sort-based group-by. Returns keys [g][nkey], count [g], sums [g][nval],
    avg [g][nval] (float64) and the overflow flags [g][nval]."""
    n = len(key_cols[0])
    nkey, nval = len(key_cols), len(values)
    kc = [np.ascontiguousarray(k) for k in key_cols]
    vals = [np.ascontiguousarray(v, dtype=np.int64) for v in values]
    vp = (ctypes.c_void_p * max(1, nval))(*[v.ctypes.data for v in vals])
    cap = n if max_groups is None else max_groups
    cap = max(cap, 1)
    keys = np.empty((cap, nkey), dtype=np.int64)
    count = np.empty(cap, dtype=np.int64)
    sums = np.empty((cap, max(nval, 1)), dtype=np.int64)
    avg = np.empty((cap, max(nval, 1)), dtype=np.float64)
    ovf = np.empty((cap, max(nval, 1)), dtype=np.uint8)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    g = lib().oc_groupby(n, _p(m), nkey, _cols(kc), nval, vp, _p(keys), _p(count), _p(sums), _p(avg),
                         _p(ovf), cap)
    if g < 0:
        raise ValueError("more groups than max_groups")
    return {"keys": keys[:g], "count": count[:g], "sums": sums[:g, :nval], "avg": avg[:g, :nval],
            "overflow": ovf[:g, :nval]}


def join_pairs(build_keys: np.ndarray, probe_keys: np.ndarray, build_mask=None, probe_mask=None,
               with_pairs: bool = True):
    """Inner equi-join. Returns (cardinality, probe_rows, build_rows) ordered by
    (probe_row, build_row)."""
    bk = np.ascontiguousarray(build_keys, dtype=np.int64)
    pk = np.ascontiguousarray(probe_keys, dtype=np.int64)
    bm = None if build_mask is None else np.ascontiguousarray(build_mask, dtype=np.uint8)
    pm = None if probe_mask is None else np.ascontiguousarray(probe_mask, dtype=np.uint8)
    total = lib().oc_join(_p(bk), len(bk), _p(bm), _p(pk), len(pk), _p(pm), None, None, 0)
    if not with_pairs:
        return total, None, None
    pr = np.empty(max(total, 1), dtype=np.int64)
    br = np.empty(max(total, 1), dtype=np.int64)
    lib().oc_join(_p(bk), len(bk), _p(bm), _p(pk), len(pk), _p(pm), _p(pr), _p(br), total)
    return total, pr[:total], br[:total]


def filter_groupby(table: Dict[str, np.ndarray], query) -> dict:
    """sigma, pi and gamma for a filter + group-by query description."""
    mask = filter_mask(table, query.preds) if query.preds else None
    vals = [project(table, e)[0] for e in query.sums]
    keys = [table[c] for c in query.key.cols]
    return groupby(keys, vals, mask)


def join_agg(dim: Dict[str, np.ndarray], fact: Dict[str, np.ndarray], query) -> dict:
    """sigma on both sides, inner join on build_key = probe_key, then group by
    the build payload with SUM/COUNT/AVG of probe-side expressions."""
    bm = filter_mask(dim, query.build_preds) if query.build_preds else None
    pm = filter_mask(fact, query.probe_preds) if query.probe_preds else None
    total, pr, br = join_pairs(dim[query.build_key], fact[query.probe_key], bm, pm)
    keys = np.ascontiguousarray(dim[query.build_payload][br])
    vals = [project(fact, e)[0][pr] for e in query.sums]
    res = groupby([keys], vals)
    res["join_rows"] = total
    return res


def partition_ids(keys: np.ndarray, bits: int) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.int64)
    out = np.empty(len(k), dtype=np.int32)
    lib().oc_partition_ids(_p(k), len(k), bits, _p(out))
    return out


def partition(keys: np.ndarray, bits: int):
    """Stable hash partition. Returns (perm, offsets[2^bits + 1])."""
    k = np.ascontiguousarray(keys, dtype=np.int64)
    perm = np.empty(max(len(k), 1), dtype=np.int64)
    offs = np.empty((1 << bits) + 1, dtype=np.int64)
    lib().oc_partition(_p(k), len(k), bits, _p(perm), _p(offs))
    return perm[:len(k)], offs


# ---------------------------------------------------------------- NULLs
# A validity map is a dict column name -> Arrow bitmap (uint8, bit r of byte
# r // 8, least significant bit first, 1 = present); a column missing from it
# has no NULLs. The semantics (SQL's) are written out in oracle.c.

def _valid_ptrs(valid, names):
    bm = [None if valid is None or valid.get(c) is None else np.ascontiguousarray(valid[c], dtype=np.uint8)
          for c in names]
    arr = (ctypes.c_void_p * max(1, len(names)))(*[None if b is None else b.ctypes.data for b in bm])
    return arr, bm


def valid_bool(bits: Optional[np.ndarray], n: int) -> np.ndarray:
    """An Arrow bitmap as one bool per row (all True when there is no bitmap)."""
    if bits is None:
        return np.ones(n, dtype=bool)
    return np.unpackbits(np.ascontiguousarray(bits, dtype=np.uint8), bitorder="little")[:n].astype(bool)


def filter_mask_nullable(table, valid, preds) -> np.ndarray:
    n = len(next(iter(table.values())))
    names = sorted({p.col for p in preds})
    cols = [np.ascontiguousarray(table[c]) for c in names]
    vp, keep = _valid_ptrs(valid, names)
    pcol = np.array([names.index(p.col) for p in preds], dtype=np.int32)
    lo = np.array([p.lo for p in preds], dtype=np.int64)
    hi = np.array([p.hi for p in preds], dtype=np.int64)
    mask = np.empty(n, dtype=np.uint8)
    lib().oc_filter_nullable(_cols(cols), vp, n, len(preds), _p(pcol), _p(lo), _p(hi), _p(mask))
    return mask


def project_nullable(table, valid, expr, n: Optional[int] = None):
    """One product expression per row under NULL semantics: (values, present),
    present one byte per row (values are 0 where absent)."""
    if n is None:
        n = len(next(iter(table.values())))
    names = sorted({f.col for f in expr if f.col is not None})
    cols = [np.ascontiguousarray(table[c]) for c in names]
    vp, keep = _valid_ptrs(valid, names)
    fcol = np.array([-1 if f.col is None else names.index(f.col) for f in expr], dtype=np.int32)
    fsign = np.array([f.sign for f in expr], dtype=np.int64)
    fadd = np.array([f.add for f in expr], dtype=np.int64)
    out = np.empty(n, dtype=np.int64)
    ok = np.empty(n, dtype=np.uint8)
    lib().oc_project_nullable(_cols(cols), vp, n, len(expr), _p(fcol), _p(fsign), _p(fadd), _p(out), _p(ok))
    return out, ok


def groupby_nullable(key: np.ndarray, key_valid: Optional[np.ndarray], values, values_valid,
                     mask: Optional[np.ndarray] = None) -> dict:
    """Group-by on one key column that may hold NULLs. values_valid[v]: one byte
    per row or None. Returns keys [g] (0 for the NULL group), key_null [g],
    count [g] = COUNT(*), and [g][nval]: sums (0 where NULL), nonnull =
    COUNT(value), avg (0 where NULL); groups in ascending key order, the NULL
    group last."""
    n = len(key)
    nval = len(values)
    k = np.ascontiguousarray(key)
    kv = None if key_valid is None else np.ascontiguousarray(key_valid, dtype=np.uint8)
    vals = [np.ascontiguousarray(v, dtype=np.int64) for v in values]
    vv = [None if x is None else np.ascontiguousarray(x, dtype=np.uint8) for x in values_valid]
    vp = (ctypes.c_void_p * max(1, nval))(*[v.ctypes.data for v in vals])
    vvp = (ctypes.c_void_p * max(1, nval))(*[None if x is None else x.ctypes.data for x in vv])
    cap = max(n, 1)
    keys = np.empty(cap, dtype=np.int64)
    key_null = np.empty(cap, dtype=np.uint8)
    count = np.empty(cap, dtype=np.int64)
    sums = np.empty((cap, max(nval, 1)), dtype=np.int64)
    nonnull = np.empty((cap, max(nval, 1)), dtype=np.int64)
    avg = np.empty((cap, max(nval, 1)), dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    g = lib().oc_groupby_nullable(n, _p(m), _cols([k])[0], _p(kv), nval, vp, vvp, _p(keys), _p(key_null),
                                  _p(count), _p(sums), _p(nonnull), _p(avg), cap)
    return {"keys": keys[:g], "key_null": key_null[:g].astype(bool), "count": count[:g], "sums": sums[:g, :nval],
            "nonnull": nonnull[:g, :nval], "avg": avg[:g, :nval]}


def filter_groupby_nullable(table, valid, query) -> dict:
    """sigma, pi and gamma under NULL semantics; the query's key has one column."""
    assert len(query.key.cols) == 1, "a key that may hold NULLs has one column"
    mask = filter_mask_nullable(table, valid, query.preds) if query.preds else None
    vals, vv = zip(*[project_nullable(table, valid, e) for e in query.sums]) if query.sums else ((), ())
    kc = query.key.cols[0]
    kbits = None if valid is None else valid.get(kc)
    return groupby_nullable(table[kc], kbits, list(vals), list(vv), mask)


def join_agg_nullable(dim, dvalid, fact, fvalid, query) -> dict:
    """join_agg under NULL semantics: NULL keys match nothing on either side; a
    NULL build payload (the group key) puts the pair in the NULL group; a NULL
    probe value makes that sum's term NULL."""
    nd = len(dim[query.build_key])
    nf = len(fact[query.probe_key])
    bm = (filter_mask_nullable(dim, dvalid, query.build_preds) if query.build_preds
          else np.ones(nd, np.uint8)).astype(bool)
    pm = (filter_mask_nullable(fact, fvalid, query.probe_preds) if query.probe_preds
          else np.ones(nf, np.uint8)).astype(bool)
    bm &= valid_bool(None if dvalid is None else dvalid.get(query.build_key), nd)
    pm &= valid_bool(None if fvalid is None else fvalid.get(query.probe_key), nf)
    total, pr, br = join_pairs(dim[query.build_key], fact[query.probe_key], bm.astype(np.uint8),
                               pm.astype(np.uint8))
    keys = np.ascontiguousarray(dim[query.build_payload][br])
    kvalid = valid_bool(None if dvalid is None else dvalid.get(query.build_payload), nd)[br]
    kbits = np.packbits(kvalid.astype(np.uint8), bitorder="little")
    vals, vv = [], []
    for e in query.sums:
        v, ok = project_nullable(fact, fvalid, e)
        vals.append(v[pr])
        vv.append(ok[pr])
    res = groupby_nullable(keys, kbits, vals, vv)
    res["join_rows"] = total
    return res


# ---------------------------------------------------------------------------
# dictionary-encoded strings (Arrow dictionary arrays, Section 3.4)

def dict_unify(build, probe) -> np.ndarray:
    """remap[i] = index of the build dictionary entry byte-equal to probe entry
    i, or -1. build/probe: (int32 offsets, uint8 data) Arrow string columns;
    the build dictionary's entries are distinct."""
    bo, bd = (np.ascontiguousarray(build[0], np.int32), np.ascontiguousarray(build[1], np.uint8))
    po, pd = (np.ascontiguousarray(probe[0], np.int32), np.ascontiguousarray(probe[1], np.uint8))
    npr = len(po) - 1
    remap = np.empty(max(npr, 1), np.int32)
    lib().oc_dict_unify(_p(bo), _p(bd), len(bo) - 1, _p(po), _p(pd), npr, _p(remap))
    return remap[:npr]


def decode(strings, codes: np.ndarray, valid: Optional[np.ndarray] = None) -> list:
    """The strings a code column stands for (None where the code is NULL)."""
    off, data = strings
    ok = valid_bool(valid, len(codes))
    out = []
    for c, v in zip(np.asarray(codes).tolist(), ok.tolist()):
        out.append(bytes(data[off[c]:off[c + 1]]) if v else None)
    return out


def join_agg_strings(build_dict, dim, dvalid, probe_dict, fact, fvalid, query) -> dict:
    """join_agg_nullable with the join keys compared as strings: both key
    columns are decoded, every distinct string gets one integer id (in order
    of first appearance), and the join runs on those ids."""
    bk = decode(build_dict, dim[query.build_key], None if dvalid is None else dvalid.get(query.build_key))
    pk = decode(probe_dict, fact[query.probe_key], None if fvalid is None else fvalid.get(query.probe_key))
    ids: Dict[bytes, int] = {}
    for s in bk + pk:
        if s is not None and s not in ids:
            ids[s] = len(ids)
    bi = np.array([0 if s is None else ids[s] for s in bk], np.int64)
    pi = np.array([0 if s is None else ids[s] for s in pk], np.int64)
    return join_agg_nullable(dict(dim, **{query.build_key: bi}), dvalid, dict(fact, **{query.probe_key: pi}),
                             fvalid, query)


def first_occurrence(strings) -> np.ndarray:
    """first[i] = the smallest row whose string equals string i's (the plain
    definition of "same dictionary entry"); strings: an (offsets, data) column."""
    off, data = strings
    n = len(off) - 1
    seen: Dict[bytes, int] = {}
    first = np.empty(n, np.int64)
    for i in range(n):
        s = bytes(data[off[i]:off[i + 1]])
        first[i] = seen.setdefault(s, i)
    return first
