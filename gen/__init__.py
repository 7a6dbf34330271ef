"""Seeded synthetic transaction databases.

This module only draws inputs: it holds none of the mining arithmetic, and both
the CPU oracle and the GPU library consume what it returns.  Every database is
returned in the transaction-list form the paper starts from (Section III: each
transaction T_i is a set of item ids), stored as CSR:

    row_ptr : uint64[n + 1]   row_ptr[0] = 0, row_ptr[n] = nnz
    col_idx : uint32[nnz]     item ids of transaction i are col_idx[row_ptr[i]:row_ptr[i+1]]

Rows produced by the named workloads are sorted and free of duplicates; the
small fuzz generator can add duplicates, unsorted rows and empty rows on purpose.

The named workloads are synthetic stand-ins for the paper's Groceries data
(Section IV-A: about 9,835 sparse baskets over 169 items) and for the classic
Quest-style benchmark shapes; no record of any public dataset is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Db", "minsup_from_ppm", "basket_zipf", "quest", "dense_planted",
    "batch_params", "batch_dbs", "make_config", "random_small", "from_rows",
    "CONFIG_NAMES",
]


@dataclasses.dataclass
class Db:
    name: str
    row_ptr: np.ndarray   # uint64[n+1]
    col_idx: np.ndarray   # uint32[nnz]
    n: int
    m: int
    minsup: int

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def minsup_from_ppm(ppm: int, n: int) -> int:
    """Absolute minimum support for a relative threshold of `ppm` parts per million.

    s = ceil(ppm * n / 1e6) in exact integer arithmetic, and at least 1, so that
    supp >= s  <=>  supp / n >= ppm / 1e6.
    """
    s = (int(ppm) * int(n) + 999_999) // 1_000_000
    return max(1, s)


def from_rows(rows, m: int | None = None, name: str = "rows", minsup: int = 1) -> Db:
    """CSR from a list of item lists (kept as given: order and duplicates preserved)."""
    lens = np.array([len(r) for r in rows], dtype=np.uint64)
    row_ptr = np.zeros(len(rows) + 1, dtype=np.uint64)
    np.cumsum(lens, out=row_ptr[1:])
    col_idx = np.array([x for r in rows for x in r], dtype=np.uint32)
    if m is None:
        m = int(col_idx.max()) + 1 if col_idx.size else 0
    return Db(name, row_ptr, col_idx, len(rows), int(m), int(minsup))


def _csr_from_pairs(rows: np.ndarray, items: np.ndarray, n: int, m: int) -> tuple[np.ndarray, np.ndarray]:
    """Sorted, de-duplicated CSR from parallel (row, item) arrays."""
    key = rows.astype(np.int64) * np.int64(m) + items.astype(np.int64)
    key = np.unique(key)
    r = (key // m).astype(np.int64)
    c = (key % m).astype(np.uint32)
    counts = np.bincount(r, minlength=n).astype(np.uint64)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, c


def _bernoulli_positions(rng: np.random.Generator, n: int, p: float) -> np.ndarray:
    """Indices i < n of a Bernoulli(p) process, drawn by geometric gaps."""
    if p <= 0.0 or n == 0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(n, dtype=np.int64)
    expect = n * p
    chunk = int(expect + 6.0 * math.sqrt(expect) + 16)
    out = []
    pos = -1
    while True:
        gaps = rng.geometric(p, size=chunk)
        idx = pos + np.cumsum(gaps)
        keep = idx[idx < n]
        out.append(keep)
        if keep.size < idx.size:
            break
        pos = int(idx[-1])
    return np.concatenate(out).astype(np.int64)


def _zipf_weights(m: int, s: float) -> np.ndarray:
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def basket_zipf(seed: int = 1, n: int = 10_000, m: int = 169, mean_extra: float = 3.4,
                cap: int = 32, zipf_s: float = 1.1, minsup_ppm: int = 10_000) -> Db:
    """Small market-basket database shaped like the paper's Groceries data.

    Row length L_i = min(1 + Poisson(mean_extra), cap); the L_i items of a row are
    drawn without replacement with weights proportional to rank^-zipf_s
    (Efraimidis-Spirakis keys log(U)/w, largest L_i keys win); a seeded
    permutation maps popularity rank to item id, so id order is not popularity.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m).astype(np.uint32)
    w = _zipf_weights(m, zipf_s)
    lens = np.minimum(1 + rng.poisson(mean_extra, size=n), min(cap, m))
    keys = np.log(rng.random((n, m))) / w[None, :]
    order = np.argsort(-keys, axis=1, kind="stable")
    take = np.arange(m)[None, :] < lens[:, None]
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    ranks = order[take]
    items = perm[ranks]
    row_ptr, col_idx = _csr_from_pairs(rows, items, n, m)
    return Db(f"basket_zipf_{n}x{m}", row_ptr, col_idx, n, m, minsup_from_ppm(minsup_ppm, n))


def quest(seed: int, n: int, m: int, mean_len: float, n_patterns: int, pat_extra: float,
          corruption: float = 0.5, zipf_s: float = 1.0, minsup_ppm: int = 2_500,
          name: str | None = None) -> Db:
    """Quest-style database: weighted corrupted patterns plus Zipf noise.

    * n_patterns patterns, length 1 + Poisson(pat_extra) (capped at m), items uniform
      without replacement; pattern weights Exp(1), normalised.
    * Row length L_i = max(1, Poisson(mean_len)); pattern budget b_i = L_i // 2.
    * Pattern instances are drawn by weight as one stream; each item of an
      instance is kept with probability 1 - corruption.  Instance j goes to the
      row whose cumulative-budget interval contains the running kept-item count
      before j, so each row receives about b_i pattern items.
    * Noise: L_i - (pattern items of row i) items drawn i.i.d. from a Zipf(zipf_s)
      law over a seeded rank->id permutation; duplicates collapse.
    """
    rng = np.random.default_rng(seed)
    # patterns
    plen = np.minimum(1 + rng.poisson(pat_extra, size=n_patterns), m).astype(np.int64)
    pat_ptr = np.zeros(n_patterns + 1, dtype=np.int64)
    np.cumsum(plen, out=pat_ptr[1:])
    pat_items = np.empty(int(pat_ptr[-1]), dtype=np.int64)
    for p in range(n_patterns):
        pat_items[pat_ptr[p]:pat_ptr[p + 1]] = rng.choice(m, size=int(plen[p]), replace=False)
    pw = rng.exponential(1.0, size=n_patterns)
    pw /= pw.sum()
    # rows
    lens = np.maximum(1, rng.poisson(mean_len, size=n)).astype(np.int64)
    budget = lens // 2
    cum_budget = np.cumsum(budget)
    total_budget = int(cum_budget[-1]) if n else 0
    # stream of pattern instances until the running kept count covers all budgets
    mean_kept = max(1e-9, float((plen * pw).sum()) * (1.0 - corruption))
    inst_pat_parts, inst_kept_parts, kept_item_parts, kept_inst_parts = [], [], [], []
    running = 0
    base = 0
    while running < total_budget:
        need = total_budget - running
        cnt = int(need / mean_kept * 1.05) + 64
        ip = rng.choice(n_patterns, size=cnt, p=pw)
        ln = plen[ip]
        starts = pat_ptr[ip]
        inst_of_item = np.repeat(np.arange(cnt, dtype=np.int64), ln)
        offs = np.arange(int(ln.sum()), dtype=np.int64) - np.repeat(np.cumsum(ln) - ln, ln)
        items = pat_items[np.repeat(starts, ln) + offs]
        keep = rng.random(items.size) >= corruption
        kept_per_inst = np.bincount(inst_of_item[keep], minlength=cnt)
        inst_pat_parts.append(ip)
        inst_kept_parts.append(kept_per_inst)
        kept_item_parts.append(items[keep])
        kept_inst_parts.append(inst_of_item[keep] + base)
        base += cnt
        running += int(kept_per_inst.sum())
    kept_per_inst = np.concatenate(inst_kept_parts) if inst_kept_parts else np.zeros(0, np.int64)
    kept_items = np.concatenate(kept_item_parts) if kept_item_parts else np.zeros(0, np.int64)
    kept_inst = np.concatenate(kept_inst_parts) if kept_inst_parts else np.zeros(0, np.int64)
    before = np.cumsum(kept_per_inst) - kept_per_inst          # running count before instance j
    inst_row = np.searchsorted(cum_budget, before, side="right")
    valid_inst = inst_row < n
    item_row = inst_row[kept_inst]
    ok = valid_inst[kept_inst]
    pat_rows = item_row[ok]
    pat_cols = kept_items[ok]
    got = np.bincount(pat_rows, minlength=n)
    # noise
    perm = rng.permutation(m).astype(np.int64)
    zw = _zipf_weights(m, zipf_s)
    nnoise = np.maximum(lens - got, 0)
    noise_rows = np.repeat(np.arange(n, dtype=np.int64), nnoise)
    noise_cols = perm[rng.choice(m, size=int(nnoise.sum()), p=zw)]
    rows = np.concatenate([pat_rows, noise_rows])
    cols = np.concatenate([pat_cols, noise_cols])
    row_ptr, col_idx = _csr_from_pairs(rows, cols, n, m)
    return Db(name or f"quest_{n}x{m}_L{mean_len:g}", row_ptr, col_idx, n, m,
              minsup_from_ppm(minsup_ppm, n))


def dense_planted(seed: int = 3, n: int = 1_000_000, m: int = 4096, p_top: float = 0.1,
                  p_bottom: float = 0.001, n_patterns: int = 500, pat_len: int = 6,
                  pat_rate: float = 0.01, minsup_ppm: int = 10_000) -> Db:
    """Dense-ish matrix: independent Bernoulli columns plus planted patterns.

    Item of popularity rank r (1..m) is present in each row independently with
    p_r = p_top * r^-alpha, alpha = ln(p_top/p_bottom)/ln(m) (so p_1 = p_top,
    p_m = p_bottom); a seeded permutation maps rank to id.  Then n_patterns
    patterns of pat_len distinct uniform items are each inserted into every row
    independently with probability pat_rate.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m).astype(np.int64)
    alpha = math.log(p_top / p_bottom) / math.log(m) if m > 1 else 0.0
    rows_parts, cols_parts = [], []
    for r in range(1, m + 1):
        p = p_top * r ** (-alpha)
        pos = _bernoulli_positions(rng, n, p)
        rows_parts.append(pos)
        cols_parts.append(np.full(pos.size, perm[r - 1], dtype=np.int64))
    for _ in range(n_patterns):
        items = rng.choice(m, size=pat_len, replace=False).astype(np.int64)
        pos = _bernoulli_positions(rng, n, pat_rate)
        rows_parts.append(np.repeat(pos, pat_len))
        cols_parts.append(np.tile(items, pos.size))
    rows = np.concatenate(rows_parts)
    cols = np.concatenate(cols_parts)
    row_ptr, col_idx = _csr_from_pairs(rows, cols, n, m)
    return Db(f"dense_planted_{n}x{m}", row_ptr, col_idx, n, m, minsup_from_ppm(minsup_ppm, n))


def batch_params(k: int) -> dict:
    """Parameters of database k (0..255) of the batched workload, drawn from seed 4000 + k."""
    rng = np.random.default_rng(4000 + k)
    n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
    m = int(rng.integers(50, 2001))
    mean_len = float(rng.uniform(5.0, 20.0))
    f = math.exp(rng.uniform(math.log(0.005), math.log(0.05)))
    ppm = int(round(f * 1e6))
    return dict(seed=4000 + k, n=n, m=m, mean_len=mean_len, ppm=ppm, n_patterns=2 * m)


def batch_db(k: int, scale: float = 1.0) -> Db:
    p = batch_params(k)
    n = max(1, int(round(p["n"] * scale)))
    return quest(p["seed"], n, p["m"], p["mean_len"], p["n_patterns"], 3.0,
                 minsup_ppm=p["ppm"], name=f"batch{k:03d}_{n}x{p['m']}")


def batch_dbs(count: int = 256, scale: float = 1.0) -> list[Db]:
    """The batched workload: `count` independent Quest-style databases of uneven size."""
    return [batch_db(k, scale) for k in range(count)]


CONFIG_NAMES = {
    1: "basket_zipf_10000x169_minsup100",
    2: "quest_T10I4D100K_100000x1000_minsup250",
    3: "dense_planted_1000000x4096_minsup10000",
    4: "batch256_quest_uneven",
    5: "quest_T40I10D1M_1000000x2000_minsup5000",
}


def make_config(k: int, scale: float = 1.0):
    """Workload k (1..5).  `scale` shrinks the row count for quick tests (1.0 = full size).

    Returns a Db, or for k == 4 a list of 256 Dbs.
    """
    if k == 1:
        return basket_zipf(seed=1, n=max(1, int(10_000 * scale)))
    if k == 2:
        return quest(2, max(1, int(100_000 * scale)), 1000, 10.0, 2000, 3.0,
                     minsup_ppm=2_500, name=CONFIG_NAMES[2])
    if k == 3:
        return dense_planted(seed=3, n=max(1, int(1_000_000 * scale)))
    if k == 4:
        return batch_dbs(256, scale)
    if k == 5:
        return quest(5, max(1, int(1_000_000 * scale)), 2000, 40.0, 2000, 9.0,
                     minsup_ppm=5_000, name=CONFIG_NAMES[5])
    raise ValueError(f"no workload {k}")


def random_small(seed: int, n: int, m: int, density: float = 0.3, dup_rate: float = 0.0,
                 shuffle: bool = False, empty_rate: float = 0.0) -> Db:
    """Tiny fuzz database: i.i.d. Bernoulli(density) cells, optional duplicates,
    unsorted rows and forced-empty rows."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        if empty_rate > 0 and rng.random() < empty_rate:
            rows.append([])
            continue
        r = [j for j in range(m) if rng.random() < density]
        if dup_rate > 0 and r:
            extra = [r[int(rng.integers(len(r)))] for _ in range(int(rng.binomial(len(r), dup_rate)))]
            r = r + extra
        if shuffle:
            rng.shuffle(r)
        rows.append(r)
    return from_rows(rows, m=m, name=f"small_s{seed}_{n}x{m}")
