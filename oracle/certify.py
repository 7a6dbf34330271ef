"""Certificate checker for a claimed frequent-itemset result, usable at any size.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A claimed list F of (itemset, support) equals the exact result for threshold s
iff all of the following hold:
  1. every itemset is non-empty, strictly ascending, in range; the list is in
     canonical (lexicographic) order without repeats;
  2. every claimed support equals the support from the definition (sequential
     intersection of the itemset's columns, Eq. 2 extended) and is >= s;
  3. F is downward closed: every (|X|-1)-subset of every X in F is in F;
  4. every set of the negative border has support < s.  The negative border is
     the set of X + {j} not in F with X in F or X empty, j not in X, and every
     |X|-subset of X + {j} in F.
If some frequent set were missing, a minimal missing one has all its proper
subsets in F, so it lies in the negative border, contradicting 4.  Hence 1-4
imply F is exactly the set of frequent itemsets with their supports.

Level-2 border sets can be checked against the closed-form pair matrix or by
intersections; `border_sample` limits the number of border sets checked (then the
certificate is a sampled one, which the caller states).
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from . import pairs as _pairs


class CertificateError(AssertionError):
    pass


def _as_list(F):
    if isinstance(F, tuple) and len(F) == 3:
        offs, items, supp = F
        offs = np.asarray(offs, dtype=np.int64)
        items = np.asarray(items)
        supp = np.asarray(supp)
        return [(tuple(int(x) for x in items[offs[i]:offs[i + 1]]), int(supp[i])) for i in range(len(offs) - 1)]
    return [(tuple(int(x) for x in X), int(v)) for X, v in F]


def _csr(sets):
    offs = np.zeros(len(sets) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(s) for s in sets]) if sets else []
    items = np.array([x for s in sets for x in s], dtype=np.uint32)
    return offs, items


def certify(orc_db, F, minsup: int, border_sample: int | None = None, seed: int = 0,
            threads: int | None = None, pair_closed_form: bool = False, csr=None) -> dict:
    """Check claimed result F against the oracle database `orc_db` (an oracle.cpp.OracleDb).

    F is a list of (itemset, support) or a tuple (offsets, items, supports).
    Returns counts of what was checked; raises CertificateError on any failure.
    """
    L = _as_list(F)
    m = orc_db.m
    s = int(minsup)
    # 1. shape and order
    prev = None
    for X, v in L:
        if len(X) == 0:
            raise CertificateError("empty itemset in result")
        if any(X[i] >= X[i + 1] for i in range(len(X) - 1)):
            raise CertificateError(f"itemset not strictly ascending: {X}")
        if X[-1] >= m:
            raise CertificateError(f"item id out of range: {X}")
        if prev is not None and not (prev < X):
            raise CertificateError(f"result not in canonical order at {prev} -> {X}")
        prev = X
    Fd = {X: v for X, v in L}
    # 2. supports
    offs, items = _csr([X for X, _ in L])
    true = orc_db.supports(offs, items, threads) if L else np.zeros(0, np.uint32)
    for (X, v), t in zip(L, true):
        if int(t) != v:
            raise CertificateError(f"wrong support for {X}: claimed {v}, true {int(t)}")
        if v < s:
            raise CertificateError(f"infrequent itemset reported: {X} support {v} < {s}")
    # 3. downward closure
    for X, _ in L:
        if len(X) >= 2:
            for i in range(len(X)):
                sub = X[:i] + X[i + 1:]
                if sub not in Fd:
                    raise CertificateError(f"{X} in result but subset {sub} missing")
    # 4. negative border
    rng = np.random.default_rng(seed)
    by_len = defaultdict(list)
    for X, _ in L:
        by_len[len(X)].append(X)
    f1 = sorted(X[0] for X in by_len.get(1, []))
    # level 1: every item outside F must be infrequent
    border1 = [(j,) for j in range(m) if (j,) not in Fd]
    # level 2: pairs of frequent items not in F
    checked = {"sets": len(L), "border_checked": 0, "border_total": 0}
    bad = []
    for j, in border1:
        if orc_db.item_support(j) >= s:
            bad.append((j,))
    checked["border_checked"] += len(border1)
    checked["border_total"] += len(border1)
    n_pairs_total = len(f1) * (len(f1) - 1) // 2 - len(by_len.get(2, []))
    checked["border_total"] += n_pairs_total
    if pair_closed_form and csr is not None and len(f1) >= 2:
        rp, ci, n = csr
        C = _pairs.pair_support(rp, ci, n, m, cols=f1)
        for a in range(len(f1)):
            for b in range(a + 1, len(f1)):
                if (f1[a], f1[b]) not in Fd and C[a, b] >= s:
                    bad.append((f1[a], f1[b]))
        checked["border_checked"] += n_pairs_total
    elif len(f1) >= 2:
        if border_sample is None or n_pairs_total <= border_sample:
            cand2 = [(f1[a], f1[b]) for a in range(len(f1)) for b in range(a + 1, len(f1))
                     if (f1[a], f1[b]) not in Fd]
        else:
            cand2 = []
            seen = set()
            tries = 0
            while len(cand2) < border_sample and tries < 50 * border_sample:
                tries += 1
                a, b = sorted(rng.choice(len(f1), size=2, replace=False))
                P = (f1[a], f1[b])
                if P not in Fd and P not in seen:
                    seen.add(P)
                    cand2.append(P)
        if cand2:
            o, it = _csr(cand2)
            sup = orc_db.supports(o, it, threads)
            bad.extend(P for P, v in zip(cand2, sup) if int(v) >= s)
        checked["border_checked"] += len(cand2)
    # levels >= 3: join sets of length k sharing a (k-1)-prefix, keep those whose
    # k-subsets are all in F, and check the ones not in F
    kmax = max(by_len) if by_len else 0
    for k in range(2, kmax + 1):
        groups = defaultdict(list)
        for X in by_len.get(k, []):
            groups[X[:-1]].append(X[-1])
        cand = []
        for pre, lasts in groups.items():
            lasts.sort()
            for i in range(len(lasts)):
                for l in range(i + 1, len(lasts)):
                    Y = pre + (lasts[i], lasts[l])
                    if Y in Fd:
                        continue
                    if all((Y[:t] + Y[t + 1:]) in Fd for t in range(len(Y))):
                        cand.append(Y)
        checked["border_total"] += len(cand)
        if border_sample is not None and len(cand) > border_sample:
            idx = rng.choice(len(cand), size=border_sample, replace=False)
            cand = [cand[i] for i in sorted(idx)]
        if cand:
            o, it = _csr(cand)
            sup = orc_db.supports(o, it, threads)
            bad.extend(Y for Y, v in zip(cand, sup) if int(v) >= s)
        checked["border_checked"] += len(cand)
    if bad:
        raise CertificateError(f"{len(bad)} frequent itemsets missing from result, e.g. {bad[:5]}")
    return checked
