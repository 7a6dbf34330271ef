"""ctypes wrapper of oracle.cpp (sorted tid-vector miner).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Build with
`python -m oracle.build` (or through the package's build entry point).
"""
from __future__ import annotations

import ctypes
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.orc_open.restype = ctypes.c_void_p
    lib.orc_open.argtypes = [_u64p, _u32p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_char_p, ctypes.c_int]
    lib.orc_close.argtypes = [ctypes.c_void_p]
    lib.orc_item_support.restype = ctypes.c_uint32
    lib.orc_item_support.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    lib.orc_frequent_items.restype = ctypes.c_uint32
    lib.orc_frequent_items.argtypes = [ctypes.c_void_p, ctypes.c_uint32, _u32p, ctypes.c_uint32]
    lib.orc_mine.restype = ctypes.c_void_p
    lib.orc_mine.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
    for f in ("orc_res_count", "orc_res_items", "orc_res_candidates"):
        getattr(lib, f).restype = ctypes.c_uint64
        getattr(lib, f).argtypes = [ctypes.c_void_p]
    lib.orc_res_copy.argtypes = [ctypes.c_void_p, _u64p, _u32p, _u32p]
    lib.orc_res_free.argtypes = [ctypes.c_void_p]
    lib.orc_support.restype = ctypes.c_uint32
    lib.orc_support.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_uint32]
    lib.orc_supports.argtypes = [ctypes.c_void_p, _u64p, _u32p, ctypes.c_uint64, _u32p, ctypes.c_int]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class OracleDb:
    """Tidsets of one transaction database."""

    def __init__(self, row_ptr, col_idx, n: int, m: int):
        lib = _load()
        self._rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        self._ci = np.ascontiguousarray(col_idx, dtype=np.uint32)
        if self._ci.size == 0:
            self._ci = np.zeros(1, dtype=np.uint32)
        err = ctypes.create_string_buffer(256)
        h = lib.orc_open(_p(self._rp, _u64p), _p(self._ci, _u32p), n, m, err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self.h = h
        self.n, self.m = n, m
        self._lib = lib

    def close(self):
        if self.h:
            self._lib.orc_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def item_support(self, j: int) -> int:
        return int(self._lib.orc_item_support(self.h, j))

    def frequent_items(self, minsup: int) -> np.ndarray:
        k = self._lib.orc_frequent_items(self.h, minsup, None, 0)
        out = np.zeros(max(k, 1), dtype=np.uint32)
        self._lib.orc_frequent_items(self.h, minsup, _p(out, _u32p), k)
        return out[:k]

    def mine_arrays(self, minsup: int, threads: int | None = None, top_first: int = 0,
                    top_last: int = 2**32 - 1):
        """(offsets u64[F+1], items u32, supports u32, candidates) in canonical order."""
        threads = default_threads() if threads is None else threads
        r = self._lib.orc_mine(self.h, minsup, threads, top_first, top_last)
        if not r:
            raise ValueError("minsup must be >= 1")
        try:
            cnt = self._lib.orc_res_count(r)
            nit = self._lib.orc_res_items(r)
            cands = self._lib.orc_res_candidates(r)
            offs = np.zeros(cnt + 1, dtype=np.uint64)
            items = np.zeros(max(nit, 1), dtype=np.uint32)
            supp = np.zeros(max(cnt, 1), dtype=np.uint32)
            self._lib.orc_res_copy(r, _p(offs, _u64p), _p(items, _u32p), _p(supp, _u32p))
        finally:
            self._lib.orc_res_free(r)
        return offs, items[:nit], supp[:cnt], int(cands)

    def mine(self, minsup: int, threads: int | None = None):
        offs, items, supp, _ = self.mine_arrays(minsup, threads)
        return arrays_to_list(offs, items, supp)

    def support(self, itemset) -> int:
        a = np.ascontiguousarray(itemset, dtype=np.uint32)
        if a.size == 0:
            return self.n
        return int(self._lib.orc_support(self.h, _p(a, _u32p), a.size))

    def supports(self, offsets, items, threads: int | None = None) -> np.ndarray:
        threads = default_threads() if threads is None else threads
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        it = np.ascontiguousarray(items, dtype=np.uint32)
        if it.size == 0:
            it = np.zeros(1, dtype=np.uint32)
        cnt = offs.size - 1
        out = np.zeros(max(cnt, 1), dtype=np.uint32)
        self._lib.orc_supports(self.h, _p(offs, _u64p), _p(it, _u32p), cnt, _p(out, _u32p), threads)
        return out[:cnt]

    def time_sample(self, minsup: int, top_first: int, top_last: int, threads: int = 1):
        """Wall time and candidate count of mining a range of top-level classes."""
        t0 = time.perf_counter()
        _, _, supp, cands = self.mine_arrays(minsup, threads, top_first, top_last)
        return time.perf_counter() - t0, cands, int(supp.size)


def arrays_to_list(offs, items, supp):
    offs = np.asarray(offs, dtype=np.int64)
    items = np.asarray(items)
    return [(tuple(int(x) for x in items[offs[i]:offs[i + 1]]), int(supp[i])) for i in range(len(offs) - 1)]
