"""Boolean-matrix frequent-itemset mining on MI355X (gfx950).

Python binding of libbm.so with the names of its C ABI (include/bm.h):

    db  = bm_build(row_ptr, col_idx, n_tx, n_items)      # Eq. 1: column bitsets on the GPU
    sup = bm_item_support(db)                             # Eq. 3: single-item supports
    C   = bm_pair_support(db, items)                      # Eq. 2: pair supports (MFMA Gram)
    res = bm_mine(db, minsup)                             # all frequent itemsets, canonical order
    offsets, items, supports = res.arrays()
    rules = bm_rules_mine(res, min_conf_ppm)              # association rules, confidence and lift

Arrays may be numpy arrays or torch tensors (host or device).  Work runs on
torch's current HIP stream unless `stream` is given.  The package has no CPU
fallback: importing it without the built library raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _bm
from ._bm import (BM_K_NAMES, FLAG_ALL_MFMA, FLAG_DEPTH_FIRST, FLAG_DFS_BLOCK_ONLY, FLAG_FP4_MFMA,
                  FLAG_GRAPH,
                  FLAG_INT8_MFMA,
                  FLAG_LEVELSYNC, FLAG_NO_MFMA, FLAG_NO_PROJECT,
                  FLAG_SHUFFLE, FLAG_TIMING, FLAG_TIMING_MAIN, FLAG_TRACE, MLP_PARAMS, BmError, BmOptions)

__all__ = [
    "bm_abi_version", "bm_build", "bm_build_batch", "bm_item_support", "bm_pair_support", "bm_mine",
    "bm_mine_ex", "bm_mine_batch", "bm_mine_blocked", "bm_set_allocator", "bm_release_cached_memory", "Db", "Result", "BmError",
    "options", "FLAG_TIMING", "FLAG_NO_MFMA", "FLAG_ALL_MFMA", "FLAG_GRAPH", "FLAG_TRACE",
    "FLAG_SHUFFLE", "FLAG_LEVELSYNC", "FLAG_FP4_MFMA", "FLAG_INT8_MFMA", "FLAG_DFS_BLOCK_ONLY",
    "FLAG_TIMING_MAIN", "FLAG_DEPTH_FIRST", "FLAG_NO_PROJECT",
    "LIB_PATH", "Model", "MLP_PARAMS", "bm_autotune",
    "autotune_cached", "options_to_dict", "options_from_dict", "shape_key", "bm_rules_mine", "Rules",
]

LIB_PATH = _bm.LIB_PATH


def bm_abi_version() -> int:
    return int(_bm.lib.bm_abi_version())


class Db:
    """A transaction database resident on the GPU as packed column bitsets."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self):
        n = ctypes.c_uint64()
        m = ctypes.c_uint32()
        w = ctypes.c_uint64()
        _bm.check(_bm.lib.bm_db_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(w)),
                  "bm_db_info")
        return int(n.value), int(m.value), int(w.value)

    def free(self):
        if self._h:
            _bm.lib.bm_db_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Result:
    """Frequent itemsets with supports, held on the GPU until copied out."""

    def __init__(self, handle):
        self._h = handle

    def info(self):
        s = ctypes.c_uint64()
        t = ctypes.c_uint64()
        k = ctypes.c_uint32()
        _bm.check(_bm.lib.bm_result_info(self._h, ctypes.byref(s), ctypes.byref(t), ctypes.byref(k)),
                  "bm_result_info")
        return int(s.value), int(t.value), int(k.value)

    def __len__(self):
        return self.info()[0]

    def arrays(self, stream=None):
        """(offsets u64[F+1], items u32[T], supports u32[F]) as host numpy arrays."""
        F, T, _ = self.info()
        offs = np.zeros(F + 1, dtype=np.uint64)
        items = np.zeros(max(T, 1), dtype=np.uint32)
        supp = np.zeros(max(F, 1), dtype=np.uint32)
        _bm.check(_bm.lib.bm_result_copy(self._h, offs.ctypes.data, items.ctypes.data,
                                         supp.ctypes.data, _bm._stream_ptr(stream)),
                  "bm_result_copy")
        return offs, items[:T], supp[:F]

    def tensors(self, device="cuda", stream=None):
        """The same three arrays copied into torch tensors on `device`."""
        import torch
        F, T, _ = self.info()
        offs = torch.empty(F + 1, dtype=torch.uint64, device=device)
        items = torch.empty(max(T, 1), dtype=torch.uint32, device=device)
        supp = torch.empty(max(F, 1), dtype=torch.uint32, device=device)
        _bm.check(_bm.lib.bm_result_copy(self._h, offs.data_ptr(), items.data_ptr(),
                                         supp.data_ptr(), _bm._stream_ptr(stream)),
                  "bm_result_copy")
        return offs, items[:T], supp[:F]

    def to_list(self):
        offs, items, supp = self.arrays()
        offs = offs.astype(np.int64)
        return [(tuple(int(x) for x in items[offs[i]:offs[i + 1]]), int(supp[i]))
                for i in range(len(offs) - 1)]

    def stats(self) -> dict:
        st = _bm.BmStats()
        _bm.check(_bm.lib.bm_result_stats(self._h, ctypes.byref(st)), "bm_result_stats")
        K = st.max_len
        return {
            "max_len": K,
            "n_frequent_items": st.n_frequent_items,
            "candidates": {k: int(st.candidates[k]) for k in range(2, _bm.BM_MAX_LEVELS + 1)
                           if st.candidates[k]},
            "frequent": {k: int(st.frequent[k]) for k in range(1, _bm.BM_MAX_LEVELS + 1)
                         if st.frequent[k]},
            "candidates_total": int(st.candidates_total),
            "frequent_total": int(st.frequent_total),
            "classes_mfma": int(st.classes_mfma),
            "classes_andpop": int(st.classes_andpop),
            "kernel_ms": {n: float(st.kernel_ms[i]) for i, n in enumerate(BM_K_NAMES)},
            "kernel_launches": {n: int(st.kernel_launches[i]) for i, n in enumerate(BM_K_NAMES)},
            "kernel_bytes": {n: float(st.kernel_bytes[i]) for i, n in enumerate(BM_K_NAMES)},
            "kernel_ops": {n: float(st.kernel_ops[i]) for i, n in enumerate(BM_K_NAMES)},
            "wall_ms": float(st.wall_ms),
            "host_syncs": int(st.host_syncs),
            "dfs_tasks": int(st.dfs_tasks),
            "mfma_form": "fp4" if st.mfma_form else "int8",
        }

    def trace(self):
        """(features float32[rows, 8], labels float32[rows]) of a BM_FLAG_TRACE call."""
        rows = ctypes.c_uint64()
        _bm.check(_bm.lib.bm_result_trace(self._h, None, None, ctypes.byref(rows)), "bm_result_trace")
        n = int(rows.value)
        f = np.zeros((max(n, 1), 8), dtype=np.float32)
        y = np.zeros(max(n, 1), dtype=np.float32)
        _bm.check(_bm.lib.bm_result_trace(self._h, f.ctypes.data, y.ctypes.data, ctypes.byref(rows)),
                  "bm_result_trace")
        return f[:n], y[:n]

    def free(self):
        if self._h:
            _bm.lib.bm_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Rules:
    """Association rules of a mining result, held on the GPU until copied out."""

    def __init__(self, handle, result):
        self._h = handle
        self._result = result

    def __len__(self):
        n = ctypes.c_uint64()
        _bm.check(_bm.lib.bm_rules_info(self._h, ctypes.byref(n)), "bm_rules_info")
        return int(n.value)

    def arrays(self, stream=None):
        """dict of host arrays: z (u64 position of Z in the result), mask (u32
        antecedent over Z's items), supp_x, supp_y, supp_z (u32), conf, lift (f64)."""
        R = len(self)
        out = {"z": np.zeros(max(R, 1), dtype=np.uint64), "mask": np.zeros(max(R, 1), dtype=np.uint32),
               "supp_x": np.zeros(max(R, 1), dtype=np.uint32),
               "supp_y": np.zeros(max(R, 1), dtype=np.uint32),
               "supp_z": np.zeros(max(R, 1), dtype=np.uint32),
               "conf": np.zeros(max(R, 1), dtype=np.float64),
               "lift": np.zeros(max(R, 1), dtype=np.float64)}
        _bm.check(_bm.lib.bm_rules_copy(self._h, *(out[k].ctypes.data for k in
                                                   ("z", "mask", "supp_x", "supp_y", "supp_z",
                                                    "conf", "lift")),
                                        _bm._stream_ptr(stream)), "bm_rules_copy")
        return {k: v[:R] for k, v in out.items()}

    def to_list(self, itemsets=None):
        """[(z, X, Y, supp_x, supp_y, supp_z, conf, lift)] with X and Y as item tuples;
        itemsets: the result's to_list() (fetched when not given)."""
        a = self.arrays()
        F = itemsets if itemsets is not None else self._result.to_list()
        out = []
        for i in range(len(a["z"])):
            zi = int(a["z"][i])
            Z = F[zi][0]
            m = int(a["mask"][i])
            X = tuple(Z[p] for p in range(len(Z)) if m >> p & 1)
            Y = tuple(Z[p] for p in range(len(Z)) if not m >> p & 1)
            out.append((zi, X, Y, int(a["supp_x"][i]), int(a["supp_y"][i]), int(a["supp_z"][i]),
                        float(a["conf"][i]), float(a["lift"][i])))
        return out

    def free(self):
        if self._h:
            _bm.lib.bm_rules_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bm_rules_mine(result: Result, min_conf_ppm: int, max_len: int = 0, stream=None) -> Rules:
    """Association rules X => Y of every itemset of `result` with
    confidence >= min_conf_ppm / 10^6 (exact integer test)."""
    h = ctypes.c_void_p()
    _bm.check(_bm.lib.bm_rules_mine(result._h, min_conf_ppm, max_len, _bm._stream_ptr(stream),
                                    ctypes.byref(h)), "bm_rules_mine")
    return Rules(h, result)


def options(flags: int = 0, mfma_min_children: int = 0, andpop_chunk_words: int = 0,
            split_words: int = 0, shuffle_seed: int = 0, dfs_threads: int = 0,
            dfs_max_words: int = 0, mfma_big_children: int = 0,
            dfs_wave_max_words: int = 0, subset_max_children: int = 0,
            dfs_arena_nodes: int = 0, project_gain: int = 0) -> BmOptions:
    o = BmOptions()
    o.flags = flags
    o.mfma_min_children = mfma_min_children
    o.andpop_chunk_words = andpop_chunk_words
    o.split_words = split_words
    o.shuffle_seed = shuffle_seed
    o.dfs_threads = dfs_threads
    o.dfs_max_words = dfs_max_words
    o.mfma_big_children = mfma_big_children
    o.dfs_wave_max_words = dfs_wave_max_words
    o.subset_max_children = subset_max_children
    o.dfs_arena_nodes = dfs_arena_nodes
    o.project_gain = project_gain
    return o


def bm_build(row_ptr, col_idx, n_tx: int, n_items: int, stream=None) -> Db:
    rp, k1 = _bm._ptr(row_ptr, np.uint64)
    ci, k2 = _bm._ptr(col_idx, np.uint32) if col_idx is not None and _bm._nelem(col_idx) else (ctypes.c_void_p(0), None)
    h = ctypes.c_void_p()
    _bm.check(_bm.lib.bm_build(rp, ci, n_tx, n_items, _bm._stream_ptr(stream), ctypes.byref(h)),
              "bm_build")
    del k1, k2
    return Db(h)


def bm_build_batch(items, stream=None) -> list:
    """Build many databases at once: items = [(row_ptr, col_idx, n_tx, n_items), ...]
    (numpy arrays or torch tensors; col_idx may be None for an empty database)."""
    n = len(items)
    if n == 0:
        return []
    keep = []
    rps = (ctypes.c_void_p * n)()
    cis = (ctypes.c_void_p * n)()
    ns = (ctypes.c_uint64 * n)()
    ms = (ctypes.c_uint32 * n)()
    for i, (rp, ci, n_tx, n_items) in enumerate(items):
        if isinstance(rp, np.ndarray):
            if len(rp) != int(n_tx) + 1:
                raise ValueError(f"database {i}: row_ptr has {len(rp)} entries, expected {n_tx + 1}")
            if isinstance(ci, np.ndarray) and len(ci) < int(rp[-1]):
                raise ValueError(f"database {i}: col_idx has {len(ci)} entries, row_ptr[n] = {rp[-1]}")
        p, k = _bm._ptr(rp, np.uint64)
        rps[i] = p.value
        keep.append(k)
        if ci is not None and _bm._nelem(ci):
            p, k = _bm._ptr(ci, np.uint32)
            cis[i] = p.value
            keep.append(k)
        ns[i] = int(n_tx)
        ms[i] = int(n_items)
    out = (ctypes.c_void_p * n)()
    _bm.check(_bm.lib.bm_build_batch(n, rps, cis, ns, ms, _bm._stream_ptr(stream), out),
              "bm_build_batch")
    del keep
    return [Db(ctypes.c_void_p(out[i])) for i in range(n)]


def bm_item_support(db: Db, stream=None) -> np.ndarray:
    _, m, _ = db.info()
    out = np.zeros(max(m, 1), dtype=np.uint32)
    _bm.check(_bm.lib.bm_item_support(db.handle, out.ctypes.data, _bm._stream_ptr(stream)),
              "bm_item_support")
    return out[:m]


def bm_pair_support(db: Db, items=None, stream=None, out=None):
    """k x k pair-support matrix of `items` (None = all items).  Returns a numpy array
    unless `out` (a uint32 torch tensor with k*k elements) is given."""
    if items is None:
        _, k, _ = db.info()
        ip, keep = ctypes.c_void_p(0), None
    else:
        ip, keep = _bm._ptr(items, np.uint32)
        k = len(items)
    if out is None:
        res = np.zeros((max(k, 1), max(k, 1)), dtype=np.uint32)
        _bm.check(_bm.lib.bm_pair_support(db.handle, ip, k, res.ctypes.data, _bm._stream_ptr(stream)),
                  "bm_pair_support")
        return res[:k, :k]
    _bm.check(_bm.lib.bm_pair_support(db.handle, ip, k, out.data_ptr(), _bm._stream_ptr(stream)),
              "bm_pair_support")
    del keep
    return out


def bm_mine(db: Db, minsup: int, stream=None) -> Result:
    h = ctypes.c_void_p()
    _bm.check(_bm.lib.bm_mine(db.handle, minsup, _bm._stream_ptr(stream), ctypes.byref(h)), "bm_mine")
    return Result(h)


def bm_mine_ex(db: Db, minsup: int, opts: BmOptions | None = None, stream=None) -> Result:
    h = ctypes.c_void_p()
    op = ctypes.byref(opts) if opts is not None else None
    _bm.check(_bm.lib.bm_mine_ex(db.handle, minsup, op, _bm._stream_ptr(stream), ctypes.byref(h)),
              "bm_mine_ex")
    return Result(h)


def bm_mine_blocked(row_ptr, col_idx, n_tx: int, n_items: int, minsup: int, block_rows: int,
                    opts: BmOptions | None = None, stream=None) -> Result:
    """Out-of-core mining of a host CSR, block_rows transactions on the device at a time."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    ci = np.ascontiguousarray(col_idx, dtype=np.uint32) if col_idx is not None else None
    h = ctypes.c_void_p()
    _bm.check(_bm.lib.bm_mine_blocked(
        rp.ctypes.data, ci.ctypes.data if ci is not None and ci.size else None, n_tx, n_items,
        minsup, block_rows, ctypes.byref(opts) if opts is not None else None,
        _bm._stream_ptr(stream), ctypes.byref(h)), "bm_mine_blocked")
    return Result(h)


def bm_mine_batch(dbs, minsups, model=None, opts: BmOptions | None = None, stream=None):
    """Mine several databases in one call (one Result per database, None entries allowed)."""
    n = len(dbs)
    if len(minsups) != n:
        raise ValueError("one minsup per database")
    arr = (ctypes.c_void_p * max(n, 1))(*[d.handle if d is not None else None for d in dbs])
    ms = (ctypes.c_uint32 * max(n, 1))(*[int(x) for x in minsups])
    out = (ctypes.c_void_p * max(n, 1))()
    op = ctypes.byref(opts) if opts is not None else None
    mh = model.handle if model is not None else None
    _bm.check(_bm.lib.bm_mine_batch(arr, ms, n, mh, op, _bm._stream_ptr(stream), out),
              "bm_mine_batch")
    return [Result(ctypes.c_void_p(out[i])) for i in range(n)]


def bm_autotune(dbs, minsups, model=None, base: BmOptions | None = None, reps: int = 3,
                stream=None):
    """(fastest BmOptions, its wall ms) for mining these databases together."""
    n = len(dbs)
    if n == 0 or len(minsups) != n:
        raise ValueError("one minsup per database, at least one database")
    arr = (ctypes.c_void_p * n)(*[d.handle if d is not None else None for d in dbs])
    ms = (ctypes.c_uint32 * n)(*[int(x) for x in minsups])
    best = BmOptions()
    best_ms = ctypes.c_double()
    _bm.check(_bm.lib.bm_autotune(arr, ms, n, model.handle if model is not None else None,
                                  ctypes.byref(base) if base is not None else None, reps,
                                  _bm._stream_ptr(stream), ctypes.byref(best),
                                  ctypes.byref(best_ms)), "bm_autotune")
    return best, float(best_ms.value)


_TUNE_FIELDS = ("flags", "mfma_min_children", "andpop_chunk_words", "split_words", "dfs_threads",
                "dfs_max_words", "mfma_big_children", "dfs_wave_max_words", "subset_max_children",
                "dfs_arena_nodes", "project_gain")


def options_to_dict(o: BmOptions) -> dict:
    return {k: int(getattr(o, k)) for k in _TUNE_FIELDS}


def options_from_dict(d: dict) -> BmOptions:
    o = BmOptions()
    for k in _TUNE_FIELDS:
        setattr(o, k, int(d.get(k, 0)))
    return o


def shape_key(dbs, minsups) -> str:
    """Cache key of a tuning problem: database count and rounded size statistics."""
    import math
    live = [(d, m) for d, m in zip(dbs, minsups) if d is not None]
    info = [d.info() for d, _ in live]
    ns = [i[0] for i in info] or [0]
    ms_ = [i[1] for i in info] or [0]
    rel = [m / max(1, i[0]) for (_, m), i in zip(live, info)] or [0]
    b = lambda x: int(round(math.log2(max(1, x)) * 2))
    return (f"n{len(dbs)}-tx{b(max(ns))}.{b(sum(ns) / len(ns))}-items{b(max(ms_))}"
            f"-minsup{b(1e6 * min(rel))}.{b(1e6 * max(rel))}")


def autotune_cached(dbs, minsups, cache_path: str, model=None, reps: int = 3, stream=None):
    """bm_autotune with a JSON cache keyed by shape_key (created or extended in place)."""
    import json
    key = shape_key(dbs, minsups)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        return options_from_dict(cache[key]["options"]), cache[key]["ms"], True
    best, ms = bm_autotune(dbs, minsups, model=model, reps=reps, stream=stream)
    cache[key] = {"options": options_to_dict(best), "ms": ms}
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)
    return best, ms, False


class Model:
    """Scheduler cost model (8 -> 64 -> 64 -> 1, BF16 weights, trained on the GPU)."""

    def __init__(self, seed: int = 0, path: str | None = None):
        h = ctypes.c_void_p()
        if path is not None:
            _bm.check(_bm.lib.bm_model_load(path.encode(), ctypes.byref(h)), "bm_model_load")
        else:
            _bm.check(_bm.lib.bm_model_create(seed, ctypes.byref(h)), "bm_model_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def save(self, path: str):
        _bm.check(_bm.lib.bm_model_save(self._h, path.encode()), "bm_model_save")

    def train(self, feats, labels, epochs: int = 20, lr: float = 1e-3, batch: int = 256,
              stream=None, graph: bool = True, all_losses: bool = False):
        """Train on the device; returns the last epoch's loss (or every epoch's)."""
        X = np.ascontiguousarray(feats, dtype=np.float32)
        Y = np.ascontiguousarray(labels, dtype=np.float32)
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        _bm.check(_bm.lib.bm_model_train_ex(
            self._h, X.ctypes.data, Y.ctypes.data, len(Y), epochs, lr, batch,
            FLAG_GRAPH if graph else 0, losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            _bm._stream_ptr(stream)), "bm_model_train_ex")
        losses = losses[:epochs]
        if all_losses:
            return losses
        return float(losses[-1]) if epochs else 0.0

    def predict(self, feats, stream=None) -> np.ndarray:
        X = np.ascontiguousarray(feats, dtype=np.float32)
        out = np.zeros(max(len(X), 1), dtype=np.float32)
        _bm.check(_bm.lib.bm_model_predict(self._h, X.ctypes.data, len(X), out.ctypes.data,
                                           _bm._stream_ptr(stream)), "bm_model_predict")
        return out[:len(X)]

    def grad(self, feats, labels, stream=None):
        X = np.ascontiguousarray(feats, dtype=np.float32)
        Y = np.ascontiguousarray(labels, dtype=np.float32)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _bm.check(_bm.lib.bm_model_grad(self._h, X.ctypes.data, Y.ctypes.data, len(Y), g.ctypes.data,
                                        ctypes.byref(loss), _bm._stream_ptr(stream)), "bm_model_grad")
        return g, float(loss.value)

    def params(self):
        """(FP32 master copy, BF16 weights as float32, normalisation [16])."""
        m = np.zeros(MLP_PARAMS, dtype=np.float32)
        w = np.zeros(MLP_PARAMS, dtype=np.float32)
        nrm = np.zeros(16, dtype=np.float32)
        _bm.check(_bm.lib.bm_model_params(self._h, m.ctypes.data, w.ctypes.data, nrm.ctypes.data),
                  "bm_model_params")
        return m, w, nrm

    def set_params(self, master=None, norm=None):
        mp = np.ascontiguousarray(master, dtype=np.float32) if master is not None else None
        npp = np.ascontiguousarray(norm, dtype=np.float32) if norm is not None else None
        _bm.check(_bm.lib.bm_model_set_params(self._h, mp.ctypes.data if mp is not None else None,
                                              npp.ctypes.data if npp is not None else None),
                  "bm_model_set_params")

    def free(self):
        if self._h:
            _bm.lib.bm_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_allocator_keepalive = None


def bm_set_allocator(alloc=None, free=None):
    """Route device allocations through Python callables alloc(size, stream) -> int pointer and
    free(ptr, stream); None, None restores the built-in pool."""
    global _allocator_keepalive
    if alloc is None and free is None:
        st = _bm.lib.bm_set_allocator(_bm.ALLOC_FN(), _bm.FREE_FN(), None)
        _bm.check(st, "bm_set_allocator")
        _allocator_keepalive = None
        return
    a = _bm.ALLOC_FN(lambda size, stream, ctx: alloc(int(size), stream) or 0)
    f = _bm.FREE_FN(lambda ptr, stream, ctx: free(int(ptr), stream))
    _bm.check(_bm.lib.bm_set_allocator(a, f, None), "bm_set_allocator")
    _allocator_keepalive = (a, f)


def bm_release_cached_memory():
    _bm.check(_bm.lib.bm_release_cached_memory(), "bm_release_cached_memory")
