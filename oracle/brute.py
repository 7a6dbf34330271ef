"""Exhaustive enumeration of every itemset (m <= 16).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Shares no logic with the tidset miners: each transaction becomes a bit mask of
its items (a row of M, Eq. 1) and the support of an itemset mask X is the number
of rows r with (r & X) == X -- the horizontal subset test, applied to all
2^m - 1 non-empty masks.
"""
from __future__ import annotations

import numpy as np


def row_masks(row_ptr, col_idx, n: int, m: int) -> np.ndarray:
    if m > 16:
        raise ValueError("brute force is limited to m <= 16")
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    masks = np.zeros(n, dtype=np.int64)
    for i in range(n):
        for j in ci[rp[i]:rp[i + 1]]:
            if j >= m:
                raise ValueError("item id out of range")
            masks[i] |= (1 << int(j))
    return masks


def all_supports(row_ptr, col_idx, n: int, m: int) -> np.ndarray:
    """supp[X] for every mask X in 0..2^m-1 (supp[0] = n)."""
    rows = row_masks(row_ptr, col_idx, n, m)
    total = 1 << m
    supp = np.zeros(total, dtype=np.int64)
    X = np.arange(total, dtype=np.int64)
    step = 256
    for a in range(0, n, step):
        r = rows[a:a + step]
        supp += ((r[:, None] & X[None, :]) == X[None, :]).sum(axis=0)
    return supp


def mine(row_ptr, col_idx, n: int, m: int, minsup: int):
    """Frequent itemsets by enumeration, canonical order."""
    supp = all_supports(row_ptr, col_idx, n, m)
    out = []
    for X in range(1, 1 << m):
        if supp[X] >= minsup:
            items = tuple(j for j in range(m) if (X >> j) & 1)
            out.append((items, int(supp[X])))
    out.sort(key=lambda e: e[0])
    return out
