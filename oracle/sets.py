"""Plain Python-set miner -- the oracle's definition of the result.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each step follows Section III of the paper:
  1. scan the transaction list and build the transactions as sets (matrix
     construction, Eq. 1; a row's duplicate ids collapse);
  2. tid[j] = { i : j in T_i } is column j of M as a set of row ids;
  3. frequent single items: |tid[j]| >= minsup (column aggregation, Eq. 3);
  4. higher orders by intersecting the prefix's row set with one more column
     at a time ("sequential AND"), recursing on frequent extensions only;
  5. the result is sorted explicitly, never trusted to come out in order.
"""
from __future__ import annotations

import math


def transactions(row_ptr, col_idx, n: int, m: int) -> list[set]:
    """Validate the CSR and return T_0..T_{n-1} as Python sets."""
    row_ptr = [int(x) for x in row_ptr]
    col_idx = [int(x) for x in col_idx]
    if len(row_ptr) != n + 1 or row_ptr[0] != 0 or row_ptr[-1] != len(col_idx):
        raise ValueError("bad row_ptr")
    out = []
    for i in range(n):
        a, b = row_ptr[i], row_ptr[i + 1]
        if b < a:
            raise ValueError("row_ptr not monotone")
        row = col_idx[a:b]
        for j in row:
            if j >= m:
                raise ValueError("item id out of range")
        out.append(set(row))
    return out


def tidsets(T: list[set], m: int) -> list[set]:
    """Column j of M as the set of transaction ids containing item j."""
    tid = [set() for _ in range(m)]
    for i, row in enumerate(T):
        for j in row:
            tid[j].add(i)
    return tid


def support(T: list[set], itemset) -> int:
    """S(X) straight from the definition: rows containing every item of X."""
    X = set(itemset)
    return sum(1 for row in T if X <= row)


def mine(row_ptr, col_idx, n: int, m: int, minsup: int, count_candidates: bool = False):
    """All frequent itemsets (support >= minsup) in canonical order.

    With count_candidates=True also returns the number of supports evaluated by
    the recursion: every (prefix, later frequent sibling) pair, i.e. sum over
    prefix classes of q(q-1)/2 with q the class's frequent extensions.
    """
    if minsup < 1:
        raise ValueError("minsup must be >= 1")
    T = transactions(row_ptr, col_idx, n, m)
    tid = tidsets(T, m)
    out = []
    counter = [0]

    def rec(prefix: tuple, cands: list):
        # cands: [(j, tidset(prefix + (j,)))], all frequent, j ascending
        for idx, (j, Tj) in enumerate(cands):
            X = prefix + (j,)
            out.append((X, len(Tj)))
            nxt = []
            for (j2, T2) in cands[idx + 1:]:
                counter[0] += 1
                inter = Tj & T2
                if len(inter) >= minsup:
                    nxt.append((j2, inter))
            if nxt:
                rec(X, nxt)

    f1 = [(j, tid[j]) for j in range(m) if len(tid[j]) >= minsup]
    rec((), f1)
    out.sort(key=lambda e: e[0])
    if count_candidates:
        return out, counter[0]
    return out


def paper_theta_to_minsup(theta) -> int:
    """The paper's criterion S(X) > theta (Eq. 3) as an absolute `>=` count."""
    return int(math.floor(theta)) + 1
