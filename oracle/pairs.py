"""Closed-form pair supports (Eq. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

S(I_a and I_b) = sum_i M[i,a] * M[i,b] for 0/1 entries, so the whole pair-support
matrix is C = M^T M.  Computed here with a library matrix product over row
blocks of the dense 0/1 matrix in float64 (every partial sum is an integer far
below 2^53, so the product is exact).
"""
from __future__ import annotations

import numpy as np


def dense_matrix(row_ptr, col_idx, n: int, m: int, r0: int = 0, r1: int | None = None,
                 cols=None, dtype=np.float64) -> np.ndarray:
    """Rows r0..r1 of M (Eq. 1) as a dense 0/1 array; optional column subset."""
    r1 = n if r1 is None else r1
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    a, b = int(rp[r0]), int(rp[r1])
    rows = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(rp[r0:r1 + 1])) - r0
    M = np.zeros((r1 - r0, m), dtype=dtype)
    M[rows, ci[a:b]] = 1
    if cols is not None:
        M = M[:, np.asarray(cols, dtype=np.int64)]
    return M


def pair_support(row_ptr, col_idx, n: int, m: int, cols=None, block: int = 65536) -> np.ndarray:
    """C[a][b] = S({cols[a], cols[b]}) (diagonal = single-item support), int64."""
    k = m if cols is None else len(cols)
    C = np.zeros((k, k), dtype=np.float64)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        A = dense_matrix(row_ptr, col_idx, n, m, r0, r1, cols)
        C += A.T @ A
    return np.rint(C).astype(np.int64)


def column_sums(row_ptr, col_idx, n: int, m: int) -> np.ndarray:
    """Single-item supports: the histogram of de-duplicated (row, item) cells."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col_idx, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    cells = np.unique(rows * max(m, 1) + ci) if ci.size else np.zeros(0, np.int64)
    return np.bincount(cells % max(m, 1), minlength=m).astype(np.int64)
