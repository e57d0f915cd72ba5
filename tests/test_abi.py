"""The C ABI without a GPU: the library loads, exports every declared entry
point, sizes buffers as documented, and rejects bad arguments before it
enqueues anything."""
import ctypes
import os
import re

import pytest

from paper_2508_05029_amd import tq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x100000  # never dereferenced: validation fails first


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            # function declarations: a name followed by "(" but not a function-pointer typedef "(*"
            names |= set(re.findall(r"\b(tq_[a-z0-9_]+)\s*\((?!\s*\*)", text)) - {"tq_status"}
    return sorted(names)


def test_every_declared_function_is_exported():
    L = tq.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = tq.lib()
    assert tq.version() >= 1
    for s in (tq.TQ_OK, tq.TQ_EINVAL, tq.TQ_ENOMEM, tq.TQ_EFULL, tq.TQ_EDOMAIN, tq.TQ_EHIP):
        assert L.tq_strerror(s)


def test_buffer_sizes():
    # 227,600 filtered dimension rows at load factor 0.5 -> 2^19 slots
    # header | partial counts | tags | slots | build scratch: rows per
    # partitioning block (one block per 2048 slots), each block's (offset,
    # count) per region, one row segment per slot, alternate tags, and the
    # Bloom filter
    part = 2048 * 8

    def scratch(cap):
        g = max(1, cap // 2048)
        bloom_words = min(max(cap // 16, 512), 32768)  # 32-bit words: two bits per slot, at most 128 KiB
        return (g * 4 + 255) // 256 * 256 + g * 264 * 4 + cap * 16 + (cap * 2 + 255) // 256 * 256 + bloom_words * 4

    assert tq.join_table_bytes(227_600, 0.5) == 256 + part + (1 << 19) * 2 + (1 << 19) * 16 + scratch(1 << 19)
    assert tq.join_table_bytes(0, 0.5) == 256 + part + 256 + 64 * 16 + scratch(64)
    assert tq.join_table_bytes(10, 0.95) == 0  # load factor above 0.9 is refused
    assert tq.groupby_state_bytes(25, 1) == 256 + 1024 * 25 * 2 * 8  # one private row per workgroup slot
    assert tq.groupby_state_bytes(65536, 1) == 256 + 65536 * 2 * 8
    assert tq.groupby_state_bytes(0, 1) == 0
    assert tq.hash_partition_scratch_bytes(4096 * 10, 8) >= 10 * 256 * 8
    assert tq.hash_partition_scratch_bytes(10, 11) == 0


def _st(v):
    return ctypes.c_void_p(v)


def test_invalid_arguments_are_rejected_synchronously():
    L = tq.lib()
    cols = tq.cols([])
    # too many columns
    S = 1 << 20
    assert L.tq_filter_project(cols, 9, 10, None, 0, None, 0, None, None, FAKE, FAKE, S, None) == tq.TQ_EINVAL
    assert b"ncol" in L.tq_last_error()
    # predicate on a column that does not exist
    c = (tq.Col * 1)(tq.Col(FAKE, tq.TQ_I64))
    assert L.tq_filter_project(c, 1, 10, tq.preds([(3, 0, 1)]), 1, None, 0, None, None, FAKE, FAKE, S,
                               None) == tq.TQ_EINVAL
    # misaligned column
    c = (tq.Col * 1)(tq.Col(FAKE + 8, tq.TQ_I64))
    assert L.tq_filter_project(c, 1, 10, None, 0, None, 0, None, None, FAKE, FAKE, S, None) == tq.TQ_EINVAL
    assert b"aligned" in L.tq_last_error()
    # bad type
    c = (tq.Col * 1)(tq.Col(FAKE, 3))
    assert L.tq_filter_project(c, 1, 10, None, 0, None, 0, None, None, FAKE, FAKE, S, None) == tq.TQ_EINVAL
    # scratch too small
    c = (tq.Col * 1)(tq.Col(FAKE, tq.TQ_I64))
    assert L.tq_filter_project(c, 1, 10, None, 0, None, 0, None, None, FAKE, FAKE, 8, None) == tq.TQ_EINVAL
    # load factor out of range, skip out of range
    pay = tq.Col(FAKE, tq.TQ_I64)
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.0, 0, 0, None) == tq.TQ_EINVAL
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 40, 0, None) == tq.TQ_EINVAL
    # one hash partition: 1 <= skip <= 16, id < 2^skip, and no id without the flag
    sel = tq.TQ_SELECT_PARTITION
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 0, sel, None) == tq.TQ_EINVAL
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 17, sel, None) == tq.TQ_EINVAL
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 2, sel | tq.TQ_PARTITION(4),
                           None) == tq.TQ_EINVAL
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 2, tq.TQ_PARTITION(1),
                           None) == tq.TQ_EINVAL
    assert L.tq_join_build(FAKE, 1 << 20, FAKE, pay, 10, None, 0, None, 0, 0.5, 0, 0x80, None) == tq.TQ_EINVAL
    # a table buffer too small for even 64 slots
    assert L.tq_join_table_init(FAKE, 100, None) == tq.TQ_EINVAL
    # the kept-row count needs a table and somewhere to write it
    r = ctypes.c_int64()
    assert L.tq_join_table_rows(None, ctypes.byref(r), None) == tq.TQ_EINVAL
    assert L.tq_join_table_rows(FAKE, None, None) == tq.TQ_EINVAL
    # group-by state: nsum, domain, size
    assert L.tq_groupby_init(FAKE, 1 << 20, 10, 7, None) == tq.TQ_EINVAL
    assert L.tq_groupby_init(FAKE, 1 << 20, 0, 1, None) == tq.TQ_EINVAL
    assert L.tq_groupby_init(FAKE, 10, 10, 1, None) == tq.TQ_EINVAL
    # partition fan-out and scratch
    assert L.tq_hash_partition(FAKE, None, 0, 10, 11, 0, FAKE, None, FAKE, FAKE, 1 << 20, None) == tq.TQ_EINVAL
    assert L.tq_hash_partition(FAKE, None, 0, 100000, 8, 0, FAKE, None, FAKE, FAKE, 16, None) == tq.TQ_EINVAL
    # the variant with the fixed scratch area: sizes beyond the area, bad fan-out
    assert tq.hash_partition_scratch_bytes(5_000_000, 10) > tq.PARTITION_STATIC_SCRATCH_BYTES
    assert L.tq_hash_partition_noalloc(FAKE, None, 0, 5_000_000, 10, 0, FAKE, None, FAKE, None) == tq.TQ_EINVAL
    assert b"fixed area" in L.tq_last_error()
    assert L.tq_hash_partition_noalloc(FAKE, None, 0, 10, 11, 0, FAKE, None, FAKE, None) == tq.TQ_EINVAL
    # dictionary strings: table, counts, NULL columns, scratch size
    S = tq.Strings
    assert L.tq_dict_unify(None, 1 << 20, S(FAKE, FAKE, 2), S(FAKE, FAKE, 2), FAKE, 1 << 20, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_unify(FAKE, 1 << 20, S(FAKE, FAKE, -1), S(FAKE, FAKE, 2), FAKE, 1 << 20, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_unify(FAKE, 1 << 20, S(None, FAKE, 2), S(FAKE, FAKE, 2), FAKE, 1 << 20, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_unify(FAKE, 1 << 20, S(FAKE, FAKE, 2), S(FAKE, FAKE, 2), FAKE, 1 << 20, None, None) == tq.TQ_EINVAL
    assert L.tq_dict_unify(FAKE, 1 << 20, S(FAKE, FAKE, 2), S(FAKE, FAKE, 2), FAKE, 16, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_keys(None, None, 5, None, 0, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_keys(FAKE, None, 5, None, 3, FAKE, None) == tq.TQ_EINVAL
    assert L.tq_dict_keys(FAKE, None, -1, None, 0, FAKE, None) == tq.TQ_EINVAL
    # probe: expression factor count
    e = tq.exprs([[(0, 1, 0)] * 3])
    e[0].nf = 4
    agg = tq.Agg(FAKE, 10, ctypes.cast(e, ctypes.POINTER(tq.ExprS)), 1)
    c = (tq.Col * 1)(tq.Col(FAKE, tq.TQ_I64))
    assert L.tq_join_probe(FAKE, FAKE, 10, c, 1, None, 0, None, None, 0, None, ctypes.byref(agg), None) == tq.TQ_EINVAL
    assert L.tq_read_peak(FAKE, 15, FAKE, None) == tq.TQ_EINVAL


def test_serving_rejects_windows_outside_the_base_tables():
    """A request window past the end of its base table is refused before any
    request runs (the kernels would otherwise read past the device columns)."""
    import torch
    T = tq.ServeTables()
    T.fg_rows, T.dim_rows, T.fact_rows = 1000, 500, 2000
    arena = torch.empty(1 << 16, dtype=torch.uint8)
    budget = tq.Budget(1 << 16)
    cases = [(0, 992, 16, 0, 0),      # filter table: rows [992, 1008) of 1000
             (1, 0, 2016, 0, 100),    # fact table: rows [0, 2016) of 2000
             (1, 0, 100, 496, 16),    # dimension: rows [496, 512) of 500
             (2, 0, 1, 496, 16)]      # the same dimension window for a streamed request
    try:
        for shape, ff, nf, df, nd in cases:
            R = (tq.Request * 1)()
            R[0].shape, R[0].fact_first, R[0].n_fact, R[0].dim_first, R[0].n_dim = shape, ff, nf, df, nd
            if shape == 2:
                T.pool, T.n_fact_batches = FAKE, 4  # a batch window that fits; never read
            with pytest.raises(tq.TqError) as e:
                tq.serve_run(T, R, 1, budget, arena, 25)
            assert e.value.status == tq.TQ_EINVAL
            assert b"outside" in tq.lib().tq_last_error(), (shape, tq.lib().tq_last_error())
    finally:
        budget.close()
