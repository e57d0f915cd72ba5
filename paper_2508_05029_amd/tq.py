"""ctypes binding of libtq.so: argument marshalling only.

Every function here has the name of a C entry point (``tq_`` dropped) and
passes torch tensor pointers and a HIP stream straight through; all the work
runs in the library's HIP kernels. Loading fails loudly if the library is not
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtq.so")

TQ_OK, TQ_EINVAL, TQ_ENOMEM, TQ_EFULL, TQ_EDOMAIN, TQ_EHIP = 0, -1, -2, -3, -4, -5
TQ_U8, TQ_I32, TQ_I64 = 1, 4, 8
TQ_UNIQUE_KEYS = 1
TQ_SELECT_PARTITION = 2


def TQ_PARTITION(i: int) -> int:
    return i << 16


MAX_COLS, MAX_PREDS, MAX_SUMS = 8, 4, 6


class TqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tq status {status}: {msg}")
        self.status = status


class Col(ctypes.Structure):
    # valid: a validity bitmap (bit r of byte r // 8, least significant first; 1 = present) or None
    _fields_ = [("data", ctypes.c_void_p), ("type", ctypes.c_int32), ("valid", ctypes.c_void_p)]


class Strings(ctypes.Structure):
    # Arrow string column: string i is data[offsets[i]:offsets[i + 1]] (int32 offsets, n + 1 of them)
    _fields_ = [("offsets", ctypes.c_void_p), ("data", ctypes.c_void_p), ("n", ctypes.c_int64)]


class PredS(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("lo", ctypes.c_int64), ("hi", ctypes.c_int64)]


class FactorS(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("sign", ctypes.c_int32), ("add", ctypes.c_int64)]


class ExprS(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int32), ("f", FactorS * 3)]


class GKey(ctypes.Structure):
    _fields_ = [("ncol", ctypes.c_int32), ("col", ctypes.c_int32 * 2), ("mult", ctypes.c_int64)]


class Agg(ctypes.Structure):
    _fields_ = [("d_state", ctypes.c_void_p), ("domain", ctypes.c_int64), ("sums", ctypes.POINTER(ExprS)),
                ("nsum", ctypes.c_int32), ("nullable", ctypes.c_int32)]


_vp, _i64, _i32, _u32, _sz, _f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                    ctypes.c_size_t, ctypes.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build(); "
                               "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "tq_strerror": (ctypes.c_char_p, [_i32]),
            "tq_last_error": (ctypes.c_char_p, []),
            "tq_version": (_i32, []),
            "tq_filter_project_scratch_bytes": (_sz, [_i64]),
            "tq_filter_project": (_i32, [_vp, _i32, _i64, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
            "tq_hash_partition_scratch_bytes": (_sz, [_i64, _i32]),
            "tq_hash_partition": (_i32, [_vp, _vp, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
            "tq_hash_partition_noalloc": (_i32, [_vp, _vp, _i32, _i64, _i32, _i32, _vp, _vp, _vp, _vp]),
            "tq_join_table_bytes": (_sz, [_i64, _f64]),
            "tq_join_table_init": (_i32, [_vp, _sz, _vp]),
            "tq_join_table_rows": (_i32, [_vp, ctypes.POINTER(ctypes.c_int64), _vp]),
            "tq_join_build": (_i32, [_vp, _sz, _vp, Col, _i64, _vp, _i32, _vp, _i32, _f64, _i32, _u32, _vp]),
            "tq_join_probe": (_i32, [_vp, _vp, _i64, _vp, _i32, _vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp]),
            "tq_groupby_state_bytes": (_sz, [_i64, _i32]),
            "tq_groupby_init": (_i32, [_vp, _sz, _i64, _i32, _vp]),
            "tq_groupby_agg": (_i32, [_vp, _i64, _vp, _i32, _i64, _vp, _i32, _vp, _vp, _i32, _vp]),
            "tq_groupby_finalize": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tq_groupby_finalize_reset": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tq_groupby_state_bytes_nullable": (_sz, [_i64, _i32]),
            "tq_groupby_init_nullable": (_i32, [_vp, _sz, _i64, _i32, _vp]),
            "tq_groupby_agg_nullable": (_i32, [_vp, _i64, _vp, _i32, _i64, _vp, _i32, _vp, _vp, _i32, _vp]),
            "tq_groupby_finalize_nullable": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tq_join_build_nullable": (_i32, [_vp, _sz, _vp, _vp, Col, _i64, _vp, _i32, _vp, _i32, _f64, _i32, _u32,
                                              _vp]),
            "tq_join_probe_nullable": (_i32, [_vp, _vp, _vp, _i64, _vp, _i32, _vp, _i32, _vp, _vp]),
            "tq_dict_unify_scratch_bytes": (_sz, [_i64]),
            "tq_dict_unify": (_i32, [_vp, _sz, Strings, Strings, _vp, _sz, _vp, _vp]),
            "tq_dict_keys": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _vp]),
            "tq_dict_encode_scratch_bytes": (_sz, [_i64]),
            "tq_dict_encode": (_i32, [Strings, _vp, _sz, _vp, _vp, _vp, _vp]),
            "tq_parquet_open": (_i32, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
            "tq_parquet_close": (None, [_vp]),
            "tq_parquet_num_rows": (_i64, [_vp]),
            "tq_parquet_num_row_groups": (_i32, [_vp]),
            "tq_parquet_row_group_rows": (_i64, [_vp, _i32]),
            "tq_parquet_num_columns": (_i32, [_vp]),
            "tq_parquet_column": (_i32, [_vp, _i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32)]),
            "tq_parquet_chunk": (_i32, [_vp, _i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                        ctypes.POINTER(_i32)]),
            "tq_parquet_preload": (_i32, [_vp, _vp, _i32, _i32, _vp, _i32, _i64, ctypes.POINTER(_vp)]),
            "tq_preload_num_reads": (_i32, [_vp]),
            "tq_preload_read": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
            "tq_preload_rows": (_i64, [_vp]),
            "tq_preload_work_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
            "tq_preload_num_pages": (_i64, [_vp]),
            "tq_preload_page": (_i32, [_vp, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                       ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
            "tq_parquet_decode": (_i32, [_vp, _vp, _sz, _vp, _vp]),
            "tq_preload_free": (None, [_vp]),
            "tq_check": (_i32, [_vp, _vp]),
            "tq_read_peak_scratch_bytes": (_sz, []),
            "tq_read_peak": (_i32, [_vp, _sz, _vp, _vp]),
            "tq_fill": (_i32, [_vp, _sz, _u32, _vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != TQ_OK:
        raise TqError(status, lib().tq_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


_TYPE = {torch.uint8: TQ_U8, torch.int32: TQ_I32, torch.int64: TQ_I64}


def cols(tensors: Sequence[torch.Tensor], valid: Optional[Sequence[Optional[torch.Tensor]]] = None):
    """Column descriptors; valid[i]: a uint8 validity bitmap tensor for column i, or None."""
    arr = (Col * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        arr[i].data = t.data_ptr()
        arr[i].type = _TYPE[t.dtype]
        if valid is not None and valid[i] is not None:
            arr[i].valid = valid[i].data_ptr()
    return arr


def col(t: torch.Tensor, valid: Optional[torch.Tensor] = None) -> Col:
    return Col(t.data_ptr(), _TYPE[t.dtype], None if valid is None else valid.data_ptr())


def preds(ps: Sequence[tuple]):
    """ps: (col_index, lo, hi) triples."""
    arr = (PredS * max(1, len(ps)))()
    for i, (c, lo, hi) in enumerate(ps):
        arr[i] = PredS(c, lo, hi)
    return arr


def exprs(es: Sequence[Sequence[tuple]]):
    """es: each a sequence of (col_index or -1, sign, add) factors."""
    arr = (ExprS * max(1, len(es)))()
    for i, e in enumerate(es):
        arr[i].nf = len(e)
        for j, (c, s, a) in enumerate(e):
            arr[i].f[j] = FactorS(c, s, a)
    return arr


def gkey(key_cols: Sequence[int], mult: int = 1) -> GKey:
    k = GKey()
    k.ncol = len(key_cols)
    k.col[0] = key_cols[0]
    k.col[1] = key_cols[1] if len(key_cols) > 1 else 0
    k.mult = mult
    return k


# ------------------------------------------------------------------ entry points

def version() -> int:
    return lib().tq_version()


def filter_project_scratch_bytes(nrows: int) -> int:
    return lib().tq_filter_project_scratch_bytes(nrows)


def filter_project(in_cols, nrows, ps, es, out, sel, out_rows, scratch, stream=None):
    E = exprs(es)
    outp = (ctypes.c_void_p * max(1, len(out)))(*[t.data_ptr() for t in out])
    _check(lib().tq_filter_project(cols(in_cols), len(in_cols), nrows, preds(ps), len(ps), E, len(es), outp,
                                   _ptr(sel), out_rows.data_ptr(), scratch.data_ptr(), _nbytes(scratch),
                                   _stream(stream)))


def hash_partition_scratch_bytes(n: int, log2_fanout: int) -> int:
    return lib().tq_hash_partition_scratch_bytes(n, log2_fanout)


def hash_partition(keys, payload, n, log2_fanout, skip, out_keys, out_payload, offsets, scratch, stream=None):
    outp = (ctypes.c_void_p * max(1, len(out_payload)))(*[t.data_ptr() for t in out_payload])
    _check(lib().tq_hash_partition(_ptr(keys), cols(payload), len(payload), n, log2_fanout, skip, _ptr(out_keys),
                                   outp, offsets.data_ptr(), _ptr(scratch),
                                   0 if scratch is None else scratch.numel() * scratch.element_size(),
                                   _stream(stream)))


def hash_partition_noalloc(keys, payload, n, log2_fanout, skip, out_keys, out_payload, offsets, stream=None):
    """tq_hash_partition with the library's fixed scratch area (no scratch argument)."""
    outp = (ctypes.c_void_p * max(1, len(out_payload)))(*[t.data_ptr() for t in out_payload])
    _check(lib().tq_hash_partition_noalloc(_ptr(keys), cols(payload), len(payload), n, log2_fanout, skip,
                                           _ptr(out_keys), outp, offsets.data_ptr(), _stream(stream)))


PARTITION_STATIC_SCRATCH_BYTES = 8 << 20  # TQ_PARTITION_STATIC_SCRATCH_BYTES


def join_table_bytes(n_build_max: int, load_factor: float) -> int:
    return lib().tq_join_table_bytes(n_build_max, load_factor)


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def join_table_init(table, stream=None):
    _check(lib().tq_join_table_init(table.data_ptr(), _nbytes(table), _stream(stream)))


def join_table_rows(table, stream=None) -> int:
    r = ctypes.c_int64()
    _check(lib().tq_join_table_rows(table.data_ptr(), ctypes.byref(r), _stream(stream)))
    return r.value


def join_build(table, keys, payload, n, filt_cols=(), ps=(), load_factor=0.5, skip=0, flags=0, stream=None):
    _check(lib().tq_join_build(table.data_ptr(), _nbytes(table), _ptr(keys), col(payload), n, cols(filt_cols),
                               len(filt_cols), preds(ps), len(ps), load_factor, skip, flags, _stream(stream)))


def join_probe(table, probe_keys, n, probe_cols=(), ps=(), out_row=None, out_payload=None, capacity=0,
               out_count=None, agg=None, stream=None):
    """agg: None, or (state, domain, exprs) for the fused group-by."""
    A = None
    if agg is not None:
        state, domain, es = agg
        E = exprs(es)
        A = Agg(state.data_ptr(), domain, ctypes.cast(E, ctypes.POINTER(ExprS)), len(es))
    _check(lib().tq_join_probe(table.data_ptr(), _ptr(probe_keys), n, cols(probe_cols), len(probe_cols), preds(ps),
                               len(ps), _ptr(out_row), _ptr(out_payload), capacity, _ptr(out_count),
                               None if A is None else ctypes.addressof(A), _stream(stream)))


def groupby_state_bytes(domain: int, nsum: int) -> int:
    return lib().tq_groupby_state_bytes(domain, nsum)


def groupby_init(state, domain, nsum, stream=None):
    _check(lib().tq_groupby_init(state.data_ptr(), _nbytes(state), domain, nsum, _stream(stream)))


def groupby_agg(state, domain, in_cols, nrows, ps, key: GKey, es, stream=None):
    _check(lib().tq_groupby_agg(state.data_ptr(), domain, cols(in_cols), len(in_cols), nrows, preds(ps), len(ps),
                                ctypes.byref(key), exprs(es), len(es), _stream(stream)))


def groupby_finalize(state, keys, count, sums, avg, ngroups, stream=None, reset=False):
    """reset=True: tq_groupby_finalize_reset (the state is left empty for the next query)."""
    fn = lib().tq_groupby_finalize_reset if reset else lib().tq_groupby_finalize
    _check(fn(state.data_ptr(), keys.data_ptr(), count.data_ptr(), sums.data_ptr(), _ptr(avg), ngroups.data_ptr(),
              _stream(stream)))


def groupby_state_bytes_nullable(domain: int, nsum: int) -> int:
    return lib().tq_groupby_state_bytes_nullable(domain, nsum)


def groupby_init_nullable(state, domain, nsum, stream=None):
    _check(lib().tq_groupby_init_nullable(state.data_ptr(), _nbytes(state), domain, nsum, _stream(stream)))


def groupby_agg_nullable(state, domain, in_cols, in_valid, nrows, ps, key: GKey, es, stream=None):
    """in_valid[i]: validity bitmap tensor of column i or None."""
    _check(lib().tq_groupby_agg_nullable(state.data_ptr(), domain, cols(in_cols, in_valid), len(in_cols), nrows,
                                         preds(ps), len(ps), ctypes.byref(key), exprs(es), len(es), _stream(stream)))


def groupby_finalize_nullable(state, keys, count, sums, nonnull, avg, ngroups, stream=None):
    _check(lib().tq_groupby_finalize_nullable(state.data_ptr(), keys.data_ptr(), count.data_ptr(), sums.data_ptr(),
                                              nonnull.data_ptr(), _ptr(avg), ngroups.data_ptr(), _stream(stream)))


def join_build_nullable(table, keys, key_valid, payload, payload_valid, n, filt_cols=(), filt_valid=None, ps=(),
                        load_factor=0.5, skip=0, flags=0, stream=None):
    _check(lib().tq_join_build_nullable(table.data_ptr(), _nbytes(table), _ptr(keys), _ptr(key_valid),
                                        col(payload, payload_valid), n, cols(filt_cols, filt_valid), len(filt_cols),
                                        preds(ps), len(ps), load_factor, skip, flags, _stream(stream)))


def join_probe_nullable(table, probe_keys, key_valid, n, probe_cols, probe_valid, ps, agg, stream=None):
    """agg: (nullable state, domain, exprs)."""
    state, domain, es = agg
    E = exprs(es)
    A = Agg(state.data_ptr(), domain, ctypes.cast(E, ctypes.POINTER(ExprS)), len(es), 1)
    _check(lib().tq_join_probe_nullable(table.data_ptr(), _ptr(probe_keys), _ptr(key_valid), n,
                                        cols(probe_cols, probe_valid), len(probe_cols), preds(ps), len(ps),
                                        ctypes.byref(A), _stream(stream)))


def strings(offsets: torch.Tensor, data: torch.Tensor) -> Strings:
    assert offsets.dtype == torch.int32 and data.dtype == torch.uint8
    return Strings(offsets.data_ptr(), data.data_ptr(), offsets.numel() - 1)


def dict_unify_scratch_bytes(n_build: int) -> int:
    return lib().tq_dict_unify_scratch_bytes(n_build)


def dict_unify(table, build, probe, scratch, remap, stream=None):
    """build/probe: (offsets, data) tensor pairs; remap: int32 tensor of probe.n entries."""
    b, p = strings(*build), strings(*probe)
    _check(lib().tq_dict_unify(table.data_ptr(), table.numel(), b, p, scratch.data_ptr(), scratch.numel(),
                               _ptr(remap), _stream(stream)))


def dict_encode_scratch_bytes(n: int) -> int:
    return lib().tq_dict_encode_scratch_bytes(n)


def dict_encode(column, scratch, codes, first_rows, ndict, stream=None):
    """column: (offsets, data) tensors; codes, first_rows: int32 tensors of n; ndict: int64 tensor of 1."""
    _check(lib().tq_dict_encode(strings(*column), scratch.data_ptr(), scratch.numel(), _ptr(codes), _ptr(first_rows),
                                ndict.data_ptr(), _stream(stream)))


def dict_keys(codes, valid, n, remap, keys, stream=None):
    nr = 0 if remap is None else remap.numel()
    _check(lib().tq_dict_keys(codes.data_ptr(), _ptr(valid), n, _ptr(remap), nr, keys.data_ptr(), _stream(stream)))


def check(obj, stream=None):
    _check(lib().tq_check(obj.data_ptr(), _stream(stream)))


def read_peak_scratch_bytes() -> int:
    return lib().tq_read_peak_scratch_bytes()


def read_peak(src, partial, stream=None):
    _check(lib().tq_read_peak(src.data_ptr(), _nbytes(src), partial.data_ptr(), _stream(stream)))


def fill(dst, pattern=0, stream=None):
    _check(lib().tq_fill(dst.data_ptr(), _nbytes(dst), pattern, _stream(stream)))


# ------------------------------------------------------------------ page pool, budget, streaming

class Batch(ctypes.Structure):
    _fields_ = [("npages", ctypes.c_int32), ("page_ids", ctypes.POINTER(ctypes.c_int32)), ("nrows", ctypes.c_int64),
                ("ncol", ctypes.c_int32), ("col_offset", ctypes.POINTER(ctypes.c_int64)),
                ("col_type", ctypes.POINTER(ctypes.c_int32))]


class OocPlan(ctypes.Structure):
    _fields_ = [("dim_key_col", ctypes.c_int32), ("dim_payload_col", ctypes.c_int32),
                ("dim_preds", ctypes.POINTER(PredS)), ("dim_np", ctypes.c_int32),
                ("fact_key_col", ctypes.c_int32), ("fact_keep_mask", ctypes.c_int32),
                ("sums", ctypes.POINTER(ExprS)), ("nsum", ctypes.c_int32), ("domain", ctypes.c_int64),
                ("log2_fanout", ctypes.c_int32), ("load_factor", ctypes.c_double), ("join_flags", ctypes.c_uint32),
                ("chunk_bytes", ctypes.c_size_t), ("nslots", ctypes.c_int32), ("exchange", ctypes.c_int32)]


class OocStats(ctypes.Structure):
    _fields_ = [("bytes_h2d", ctypes.c_int64), ("bytes_d2h", ctypes.c_int64), ("spilled_chunks", ctypes.c_int64),
                ("reloaded_chunks", ctypes.c_int64), ("dim_rows_kept", ctypes.c_int64), ("fact_rows", ctypes.c_int64),
                ("peak_budget_bytes", ctypes.c_int64), ("ms_pass1", ctypes.c_double), ("ms_pass2", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("exchange", ctypes.c_int32), ("dim_restreams", ctypes.c_int32),
                ("est_dim_rows", ctypes.c_int64), ("est_from_rows", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


BATCH_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Col), ctypes.c_int32,
                            ctypes.c_int64, ctypes.c_void_p)
TQ_POOL_PAGEABLE = 1
TQ_EXCHANGE_AUTO, TQ_EXCHANGE_PARTITIONED, TQ_EXCHANGE_SINGLE = 0, 1, 2
EXCHANGE_MODES = {"auto": TQ_EXCHANGE_AUTO, "partitioned": TQ_EXCHANGE_PARTITIONED, "single": TQ_EXCHANGE_SINGLE}

_more_sig = {
    "tq_pagepool_create": (_i32, [_sz, _i64, _u32, ctypes.POINTER(ctypes.c_void_p)]),
    "tq_pagepool_destroy": (None, [_vp]),
    "tq_pagepool_alloc": (_i32, [_vp, _i64, _vp]),
    "tq_pagepool_free": (None, [_vp, _vp, _i64]),
    "tq_pagepool_page": (_vp, [_vp, _i32]),
    "tq_pagepool_free_pages": (_i64, [_vp]),
    "tq_pagepool_page_bytes": (_sz, [_vp]),
    "tq_batch_layout": (_i32, [_i64, _i32, _vp, _sz, _vp, ctypes.POINTER(_sz), ctypes.POINTER(_i64)]),
    "tq_pagepool_stream": (_i32, [_vp, _vp, _i64, _vp, _sz, _i32, BATCH_FN, _vp, _vp, _vp]),
    "tq_budget_create": (_i32, [_sz, ctypes.POINTER(ctypes.c_void_p)]),
    "tq_budget_destroy": (None, [_vp]),
    "tq_budget_reserve": (_i32, [_vp, _sz]),
    "tq_budget_release": (None, [_vp, _sz]),
    "tq_budget_used": (_sz, [_vp]),
    "tq_budget_peak": (_sz, [_vp]),
    "tq_budget_cap": (_sz, [_vp]),
    "tq_ooc_join_agg": (_i32, [_vp, _vp, _i64, _vp, _i64, ctypes.POINTER(OocPlan), _vp, _vp, _sz, _vp,
                               ctypes.POINTER(OocStats), _vp, _vp]),
}


def _bind_more():
    L = lib()
    if getattr(L, "_more_bound", False):
        return L
    for name, (res, args) in _more_sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    L._more_bound = True
    return L


class PagePool:
    """Fixed-size page-locked host pages, allocated once (tq_pagepool_*)."""

    def __init__(self, page_bytes: int, n_pages: int, pinned: bool = True):
        L = _bind_more()
        h = ctypes.c_void_p()
        _check(L.tq_pagepool_create(page_bytes, n_pages, 0 if pinned else TQ_POOL_PAGEABLE, ctypes.byref(h)))
        self.h = h
        self.page_bytes = page_bytes
        self.n_pages = n_pages

    def alloc(self, n: int):
        ids = (ctypes.c_int32 * max(1, n))()
        _check(_bind_more().tq_pagepool_alloc(self.h, n, ids))
        return [ids[i] for i in range(n)]

    def free(self, ids):
        arr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
        _bind_more().tq_pagepool_free(self.h, arr, len(ids))

    def page(self, pid: int) -> int:
        return _bind_more().tq_pagepool_page(self.h, pid) or 0

    def free_pages(self) -> int:
        return _bind_more().tq_pagepool_free_pages(self.h)

    def close(self):
        if self.h:
            _bind_more().tq_pagepool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_layout(nrows: int, types, page_bytes: int):
    t = (ctypes.c_int32 * max(1, len(types)))(*types)
    offs = (ctypes.c_int64 * max(1, len(types)))()
    nbytes = _sz()
    npages = _i64()
    _check(_bind_more().tq_batch_layout(nrows, len(types), t, page_bytes, offs, ctypes.byref(nbytes),
                                        ctypes.byref(npages)))
    return [offs[i] for i in range(len(types))], nbytes.value, npages.value


def pagepool_stream(pool: PagePool, batches, staging, nslots, fn, copy_stream=None, compute_stream=None):
    """fn(batch_idx, cols: list[(ptr, type)], nrows, compute_stream_handle) -> status; runs on this thread."""
    def cb(_user, idx, cols, ncol, nrows, stream):
        try:
            return fn(idx, [(cols[i].data, cols[i].type) for i in range(ncol)], nrows, stream) or 0
        except Exception:  # the error crosses the C boundary as a status
            return TQ_EINVAL
    c = BATCH_FN(cb)
    arr, _keep = batches
    _check(_bind_more().tq_pagepool_stream(pool.h, arr, len(arr), staging.data_ptr(), _nbytes(staging), nslots, c,
                                           None, _stream(copy_stream), _stream(compute_stream)))


class Budget:
    def __init__(self, cap_bytes: int):
        h = ctypes.c_void_p()
        _check(_bind_more().tq_budget_create(cap_bytes, ctypes.byref(h)))
        self.h = h

    def reserve(self, n):
        _check(_bind_more().tq_budget_reserve(self.h, n))

    def try_reserve(self, n) -> bool:
        return _bind_more().tq_budget_reserve(self.h, n) == TQ_OK

    def release(self, n):
        _bind_more().tq_budget_release(self.h, n)

    @property
    def used(self):
        return _bind_more().tq_budget_used(self.h)

    @property
    def peak(self):
        return _bind_more().tq_budget_peak(self.h)

    @property
    def cap(self):
        return _bind_more().tq_budget_cap(self.h)

    def close(self):
        if self.h:
            _bind_more().tq_budget_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ooc_join_agg(pool, dim_batches, fact_batches, plan: OocPlan, budget: Budget, work, state, copy_stream=None,
                 compute_stream=None) -> OocStats:
    st = OocStats()
    d_arr, _ = dim_batches
    f_arr, _ = fact_batches
    _check(_bind_more().tq_ooc_join_agg(pool.h, d_arr, len(d_arr), f_arr, len(f_arr), ctypes.byref(plan), budget.h,
                                        work.data_ptr(), _nbytes(work), state.data_ptr(), ctypes.byref(st),
                                        _stream(copy_stream), _stream(compute_stream)))
    return st


# ------------------------------------------------------------------ batched instances

class BatchQuery(ctypes.Structure):
    _fields_ = [("dim_types", ctypes.c_int32 * 4), ("ndim", ctypes.c_int32), ("preds", PredS * 2),
                ("np", ctypes.c_int32), ("fact_types", ctypes.c_int32 * 4), ("nfact", ctypes.c_int32),
                ("sums", ExprS * 2), ("nsum", ctypes.c_int32), ("join_flags", ctypes.c_uint32)]


class Instance(ctypes.Structure):
    _fields_ = [("dim_cols", ctypes.c_void_p * 4), ("n_dim", ctypes.c_int64), ("fact_cols", ctypes.c_void_p * 4),
                ("n_fact", ctypes.c_int64), ("domain", ctypes.c_int64), ("d_table", ctypes.c_void_p),
                ("table_bytes", ctypes.c_size_t), ("d_state", ctypes.c_void_p), ("state_bytes", ctypes.c_size_t),
                ("d_keys", ctypes.c_void_p), ("d_count", ctypes.c_void_p), ("d_sums", ctypes.c_void_p),
                ("d_avg", ctypes.c_void_p), ("d_ngroups", ctypes.c_void_p), ("load_factor", ctypes.c_double),
                ("build_tile", ctypes.c_int32), ("probe_tile", ctypes.c_int32)]


_batched_sig = {
    "tq_batched_state_bytes": (_sz, [_i64, _i32]),
    "tq_batched_work_bytes": (_sz, [_vp, _i32]),
    "tq_batched_prepare": (_i32, [ctypes.POINTER(BatchQuery), _vp, _i32, _vp, _sz, _vp]),
    "tq_batched_run": (_i32, [ctypes.POINTER(BatchQuery), _vp, _i32, _vp]),
    "tq_batched_check": (_i32, [_vp, _vp]),
    "tq_batched_run_per_instance": (_i32, [ctypes.POINTER(BatchQuery), _vp, _i32, _vp]),
}


def _bind_batched():
    L = lib()
    if getattr(L, "_batched_bound", False):
        return L
    for name, (res, args) in _batched_sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    L._batched_bound = True
    return L


def batched_state_bytes(domain: int, nsum: int) -> int:
    return _bind_batched().tq_batched_state_bytes(domain, nsum)


def batched_work_bytes(insts) -> int:
    return _bind_batched().tq_batched_work_bytes(insts, len(insts))


def batched_prepare(q: BatchQuery, insts, work, stream=None):
    _check(_bind_batched().tq_batched_prepare(ctypes.byref(q), insts, len(insts), work.data_ptr(), _nbytes(work),
                                              _stream(stream)))


def batched_run(q: BatchQuery, work, n: int, stream=None):
    _check(_bind_batched().tq_batched_run(ctypes.byref(q), work.data_ptr(), n, _stream(stream)))


def batched_check(work, stream=None):
    _check(_bind_batched().tq_batched_check(work.data_ptr(), _stream(stream)))


def batched_run_per_instance(q: BatchQuery, insts, stream=None):
    _check(_bind_batched().tq_batched_run_per_instance(ctypes.byref(q), insts, len(insts), _stream(stream)))


# ------------------------------------------------------------------ serving

class ServeTables(ctypes.Structure):
    _fields_ = [("fg_cols", Col * MAX_COLS), ("fg_ncol", ctypes.c_int32), ("fg_preds", PredS * MAX_PREDS),
                ("fg_np", ctypes.c_int32), ("fg_key", GKey), ("fg_sums", ExprS * MAX_SUMS), ("fg_nsum", ctypes.c_int32),
                ("fg_domain", ctypes.c_int64), ("dim_cols", Col * 4), ("dim_ncol", ctypes.c_int32),
                ("dim_preds", PredS * 2), ("dim_np", ctypes.c_int32), ("fact_cols", Col * 4),
                ("fact_ncol", ctypes.c_int32), ("join_sums", ExprS * 2), ("join_nsum", ctypes.c_int32),
                ("join_domain", ctypes.c_int64), ("load_factor", ctypes.c_double), ("pool", ctypes.c_void_p),
                ("fact_batches", ctypes.c_void_p), ("n_fact_batches", ctypes.c_int64), ("fact_map", ctypes.c_int32 * 4),
                ("nslots", ctypes.c_int32), ("estimate", ctypes.c_int32), ("fg_rows", ctypes.c_int64),
                ("dim_rows", ctypes.c_int64), ("fact_rows", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("fact_first", ctypes.c_int64), ("n_fact", ctypes.c_int64),
                ("dim_first", ctypes.c_int64), ("n_dim", ctypes.c_int64), ("arrival_s", ctypes.c_double)]


class RequestResult(ctypes.Structure):
    _fields_ = [("start_s", ctypes.c_double), ("end_s", ctypes.c_double), ("status", ctypes.c_int32),
                ("worker", ctypes.c_int32), ("ngroups", ctypes.c_int64), ("reserved_bytes", ctypes.c_int64),
                ("retries", ctypes.c_int32), ("splits", ctypes.c_int32)]


def serve_run(tables: ServeTables, reqs, workers: int, budget: Budget, arena, max_groups: int):
    import numpy as np
    L = lib()
    if not getattr(L, "_serve_bound", False):
        L.tq_serve_run.restype = _i32
        L.tq_serve_run.argtypes = [ctypes.POINTER(ServeTables), _vp, _i64, _i32, _vp, _vp, _sz, _i64, _vp, _vp, _vp,
                                   _vp, _vp]
        L._serve_bound = True
    n = len(reqs)
    keys = np.zeros((max(n, 1), max_groups), np.int64)
    count = np.zeros((max(n, 1), max_groups), np.int64)
    sums = np.zeros((max(n, 1), max_groups, MAX_SUMS), np.int64)
    avg = np.zeros((max(n, 1), max_groups, MAX_SUMS), np.float64)
    res = (RequestResult * max(n, 1))()
    _check(L.tq_serve_run(ctypes.byref(tables), reqs, n, workers, budget.h, arena.data_ptr(), _nbytes(arena), max_groups,
                          keys.ctypes.data, count.ctypes.data, sums.ctypes.data, avg.ctypes.data, res))
    return res, keys, count, sums, avg


# ----------------------------------------------------------------- Parquet scan

class ParquetFile:
    """tq_parquet_open and the metadata queries (host only)."""

    def __init__(self, path: str):
        h = ctypes.c_void_p()
        _check(lib().tq_parquet_open(path.encode(), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().tq_parquet_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_rows(self) -> int:
        return lib().tq_parquet_num_rows(self.h)

    @property
    def num_row_groups(self) -> int:
        return lib().tq_parquet_num_row_groups(self.h)

    def row_group_rows(self, rg: int) -> int:
        return lib().tq_parquet_row_group_rows(self.h, rg)

    def columns(self):
        """[(name, type, nullable)] with type TQ_I32 / TQ_I64 (0: not decodable)."""
        out = []
        for c in range(lib().tq_parquet_num_columns(self.h)):
            name, t, nl = ctypes.c_char_p(), _i32(), _i32()
            _check(lib().tq_parquet_column(self.h, c, ctypes.byref(name), ctypes.byref(t), ctypes.byref(nl)))
            out.append((name.value.decode(), t.value, bool(nl.value)))
        return out

    def chunk(self, rg: int, c: int):
        off, n, codec = _i64(), _i64(), _i32()
        _check(lib().tq_parquet_chunk(self.h, rg, c, ctypes.byref(off), ctypes.byref(n), ctypes.byref(codec)))
        return off.value, n.value, codec.value

    def preload(self, pool, rg0: int, rg1: int, cols: Sequence[int], merge_gap: int = 1 << 20) -> "Preload":
        arr = (ctypes.c_int32 * max(1, len(cols)))(*cols)
        h = ctypes.c_void_p()
        _check(lib().tq_parquet_preload(self.h, getattr(pool, "h", pool), rg0, rg1, arr, len(cols), merge_gap,
                                        ctypes.byref(h)))
        return Preload(h, self)


class Preload:
    """tq_preload: the reads under way, the page walk, the decode."""

    def __init__(self, h, owner):
        self.h = h
        self.owner = owner  # keeps the file open while the reads run

    def reads(self):
        out = []
        for i in range(lib().tq_preload_num_reads(self.h)):
            off, n = _i64(), _i64()
            _check(lib().tq_preload_read(self.h, i, ctypes.byref(off), ctypes.byref(n)))
            out.append((off.value, n.value))
        return out

    @property
    def rows(self) -> int:
        return lib().tq_preload_rows(self.h)

    def work_bytes(self) -> int:
        n = _sz()
        _check(lib().tq_preload_work_bytes(self.h, ctypes.byref(n)))
        return n.value

    def pages(self):
        """[(row0, nrows, col, kind, encoding)] after work_bytes()."""
        out = []
        for i in range(lib().tq_preload_num_pages(self.h)):
            r0, nr, c, k, e = _i64(), _i32(), _i32(), _i32(), _i32()
            _check(lib().tq_preload_page(self.h, i, ctypes.byref(r0), ctypes.byref(nr), ctypes.byref(c),
                                         ctypes.byref(k), ctypes.byref(e)))
            out.append((r0.value, nr.value, c.value, k.value, e.value))
        return out

    def decode(self, work, out_cols, stream=None):
        """out_cols: [(data tensor, valid tensor or None)] in the preload's column order."""
        arr = cols([d for d, _ in out_cols], [v for _, v in out_cols])
        _check(lib().tq_parquet_decode(self.h, work.data_ptr(), _nbytes(work), arr, _stream(stream)))

    def free(self):
        if self.h:
            lib().tq_preload_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
