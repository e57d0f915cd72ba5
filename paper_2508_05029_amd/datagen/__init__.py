"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws input columns; it holds none of the query arithmetic.
The C kernels live in ``datagen.c`` (built into ``libtqgen.so`` beside this
file). Every value is a pure function of (seed, stream, row index), so a table
can be generated whole or batch by batch with identical contents.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtqgen.so")
_lib = None

_i64, _u64, _f64, _vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        for name in ("tg_uniform_i64", "tg_uniform_i32", "tg_uniform_u8"):
            getattr(L, name).argtypes = [_vp, _i64, _u64, _u64, _i64, _i64, _i64]
        L.tg_sequence_i64.argtypes = [_vp, _i64, _i64]
        L.tg_permutation_i64.argtypes = [_vp, _i64, _i64, _u64, _u64, _i64, _i64]
        L.tg_zipf_cdf.argtypes = [_vp, _i64, _f64]
        L.tg_zipf_i64.argtypes = [_vp, _i64, _vp, _i64, _u64, _u64, _i64]
        L.tg_log_uniform_i64.argtypes = [_vp, _i64, _f64, _f64, _i64, _i64, _u64, _u64]
        L.tg_log2_uniform_i64.argtypes = [_vp, _i64, _f64, _f64, _i64, _i64, _u64, _u64]
        L.tg_exponential_f64.argtypes = [_vp, _i64, _f64, _u64, _u64]
        L.tg_unit_f64.argtypes = [_vp, _i64, _u64, _u64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


_FILL = {np.dtype(np.int64): "tg_uniform_i64", np.dtype(np.int32): "tg_uniform_i32",
         np.dtype(np.uint8): "tg_uniform_u8"}


def uniform_into(addr: int, dtype, n: int, lo: int, hi: int, seed: int, stream: int, first: int = 0):
    """Fill raw memory at ``addr`` with n draws of U{lo..hi} for rows first..first+n-1."""
    getattr(lib(), _FILL[np.dtype(dtype)])(addr, n, seed, stream, lo, hi, first)


def uniform(n: int, lo: int, hi: int, dtype=np.int64, seed: int = 0, stream: int = 0, first: int = 0):
    out = np.empty(n, dtype=dtype)
    if n:
        uniform_into(_ptr(out), dtype, n, lo, hi, seed, stream, first)
    return out


def sequence(n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    if n:
        lib().tg_sequence_i64(_ptr(out), n, start)
    return out


def permutation_into(addr: int, count: int, n: int, seed: int, stream: int, first: int = 0, offset: int = 0):
    lib().tg_permutation_i64(addr, count, n, seed, stream, first, offset)


def permutation(n: int, seed: int = 0, stream: int = 0, offset: int = 0) -> np.ndarray:
    """A keyed permutation of offset + [0, n)."""
    out = np.empty(n, dtype=np.int64)
    if n:
        permutation_into(_ptr(out), n, n, seed, stream, 0, offset)
    return out


def zipf_cdf(G: int, s: float) -> np.ndarray:
    cdf = np.empty(G, dtype=np.float64)
    lib().tg_zipf_cdf(_ptr(cdf), G, s)
    return cdf


def zipf(n: int, G: int, s: float, seed: int = 0, stream: int = 0, cdf=None, first: int = 0):
    """Zipf(s) ranks over 1..G, returned as rank - 1 (0 is the hottest value)."""
    if cdf is None:
        cdf = zipf_cdf(G, s)
    out = np.empty(n, dtype=np.int64)
    if n:
        lib().tg_zipf_i64(_ptr(out), n, _ptr(cdf), G, seed, stream, first)
    return out


def log_uniform(n: int, a: float, b: float, lo: int, hi: int, seed: int, stream: int) -> np.ndarray:
    """floor(10^(a + (b - a) U)) clamped to [lo, hi]."""
    out = np.empty(n, dtype=np.int64)
    lib().tg_log_uniform_i64(_ptr(out), n, a, b, lo, hi, seed, stream)
    return out


def log2_uniform(n: int, base: float, e: float, lo: int, hi: int, seed: int, stream: int) -> np.ndarray:
    """floor(base * 2^(e U)) clamped to [lo, hi]."""
    out = np.empty(n, dtype=np.int64)
    lib().tg_log2_uniform_i64(_ptr(out), n, base, e, lo, hi, seed, stream)
    return out


def exponential(n: int, lam: float, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().tg_exponential_f64(_ptr(out), n, lam, seed, stream)
    return out


def unit(n: int, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().tg_unit_f64(_ptr(out), n, seed, stream)
    return out
