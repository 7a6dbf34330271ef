"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library.  Each oracle function is checked against
something other than itself: brute-force enumeration, closed forms, identities,
special cases with known answers, a hand-derived worked example and
certificate conditions.  The mutation tests at the end plant plausible mistakes
in a copy of the Python oracle and check that the pins catch each of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import gen
from oracle import brute, certify, pairs, sets
from oracle import cpp as ocpp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_hand_example():
    rows, F, C, theta = [], [], {}, {}
    n = m = minsup = None
    with open(os.path.join(GOLDEN, "hand_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "n":
                n, m = int(tok[1]), int(tok[3])
            elif tok[0] == "minsup":
                minsup = int(tok[1])
            elif tok[0] == "T":
                rows.append([int(x) for x in tok[1:]])
            elif tok[0] == "F":
                k = tok.index(":")
                F.append((tuple(int(x) for x in tok[1:k]), int(tok[k + 1])))
            elif tok[0] == "C":
                C[int(tok[1])] = int(tok[2])
            elif tok[0] == "THETA":
                theta[int(tok[1])] = int(tok[2])
    db = gen.from_rows(rows, m=m, minsup=minsup)
    assert db.n == n
    return db, F, C, theta


def run_all(db, minsup):
    return (
        sets.mine(db.row_ptr, db.col_idx, db.n, db.m, minsup),
        ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(minsup, threads=2),
    )


# ---------------------------------------------------------------- worked example

def test_hand_example_sets_oracle():
    db, F, C, theta = load_hand_example()
    got, cands = sets.mine(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, count_candidates=True)
    assert got == F
    assert cands == sum(C.values())


def test_hand_example_cpp_oracle():
    db, F, C, _ = load_hand_example()
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    offs, items, supp, cands = o.mine_arrays(db.minsup, threads=3)
    assert ocpp.arrays_to_list(offs, items, supp) == F
    assert cands == sum(C.values())


def test_hand_example_brute():
    db, F, _, _ = load_hand_example()
    assert brute.mine(db.row_ptr, db.col_idx, db.n, db.m, db.minsup) == F


def test_hand_example_strict_theta():
    """The paper's S(X) > theta equals `>= floor(theta)+1`; the two thresholds differ
    exactly by the sets whose support equals theta."""
    db, F, _, theta = load_hand_example()
    for t, count in theta.items():
        s = sets.paper_theta_to_minsup(t)
        got = sets.mine(db.row_ptr, db.col_idx, db.n, db.m, s)
        assert len(got) == count
        assert [x for x in F if x[1] > t] == got
        assert sorted(set(F) - set(got)) == sorted(x for x in F if x[1] == t)
    assert sets.paper_theta_to_minsup(2.5) == 3
    assert sets.paper_theta_to_minsup(0) == 1


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_oracles_match_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(1, 11))
    n = int(rng.integers(1, 120))
    db = gen.random_small(seed, n, m, density=float(rng.uniform(0.1, 0.8)),
                          dup_rate=0.3 if seed % 3 == 0 else 0.0, shuffle=seed % 2 == 0,
                          empty_rate=0.1 if seed % 4 == 1 else 0.0)
    supp_all = brute.all_supports(db.row_ptr, db.col_idx, db.n, db.m)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    for minsup in sorted({1, 2, 3, max(1, n // 4), max(1, n // 2), n, n + 1}):
        want = brute.mine(db.row_ptr, db.col_idx, db.n, db.m, minsup)
        assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, minsup) == want
        assert o.mine(minsup, threads=2) == want
        # brute-force list is exactly the masks with enough support
        assert len(want) == int((supp_all[1:] >= minsup).sum())


def test_brute_force_subset_test_on_single_row():
    """One transaction T with minsup 1: the frequent sets are the 2^|T|-1 non-empty
    subsets of T, each with support 1."""
    T = [0, 2, 3, 5]
    db = gen.from_rows([T], m=7)
    want = sorted((c, 1) for k in range(1, len(T) + 1) for c in itertools.combinations(T, k))
    assert brute.mine(db.row_ptr, db.col_idx, db.n, db.m, 1) == want
    assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 1) == want
    assert ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(1) == want
    assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 2) == []


def test_identical_rows_power_set():
    """k identical rows T: every non-empty subset of T has support k."""
    T, k = [1, 4, 6], 7
    db = gen.from_rows([T] * k + [[0], [2, 3]], m=8)
    want = sorted((c, k) for r in range(1, 4) for c in itertools.combinations(T, r))
    for s in (3, k):
        assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, s) == want
        assert ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(s) == want


def test_minsup_n_gives_subsets_of_intersection():
    rows = [[0, 1, 2, 5], [1, 2, 5, 7], [1, 2, 3, 5], [5, 2, 1]]
    db = gen.from_rows(rows, m=8)
    inter = sorted(set.intersection(*map(set, rows)))
    want = sorted((c, 4) for r in range(1, len(inter) + 1) for c in itertools.combinations(inter, r))
    assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 4) == want
    assert ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(4) == want
    assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 5) == []
    assert ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(5) == []


def test_empty_inputs():
    for db in (gen.from_rows([], m=0), gen.from_rows([], m=5), gen.from_rows([[], [], []], m=3)):
        assert sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 1) == []
        assert ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(1) == []


def test_minsup_zero_rejected():
    db = gen.from_rows([[0]], m=1)
    with pytest.raises(ValueError):
        sets.mine(db.row_ptr, db.col_idx, db.n, db.m, 0)
    with pytest.raises(ValueError):
        ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(0)


def test_bad_csr_rejected():
    rp = np.array([0, 2, 1], dtype=np.uint64)
    ci = np.array([0, 1], dtype=np.uint32)
    with pytest.raises(ValueError):
        ocpp.OracleDb(rp, ci, 2, 3)
    with pytest.raises(ValueError):
        sets.transactions(rp, ci, 2, 3)
    rp = np.array([0, 2], dtype=np.uint64)
    ci = np.array([0, 3], dtype=np.uint32)
    with pytest.raises(ValueError):
        ocpp.OracleDb(rp, ci, 1, 3)
    with pytest.raises(ValueError):
        sets.transactions(rp, ci, 1, 3)


# ---------------------------------------------------------------- closed forms

def test_singletons_equal_column_sums():
    db = gen.make_config(1)
    colsum = pairs.column_sums(db.row_ptr, db.col_idx, db.n, db.m)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    assert [o.item_support(j) for j in range(db.m)] == colsum.tolist()
    F = sets.mine(db.row_ptr, db.col_idx, db.n, db.m, db.minsup)
    for X, v in F:
        if len(X) == 1:
            assert v == colsum[X[0]]
    assert {X[0] for X, _ in F if len(X) == 1} == {j for j in range(db.m) if colsum[j] >= db.minsup}


def test_column_sums_collapse_duplicates():
    db = gen.from_rows([[1, 1, 2], [2, 2, 2], [0]], m=3)
    assert pairs.column_sums(db.row_ptr, db.col_idx, db.n, db.m).tolist() == [1, 1, 2]
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    assert [o.item_support(j) for j in range(3)] == [1, 1, 2]


def test_pair_supports_equal_gram_matrix():
    """Eq. 2 in matrix form: the pair-support matrix is M^T M.  The oracle's
    intersection supports must equal an independent dense product of the 0/1
    matrix (computed here in int64 without the oracle)."""
    db = gen.make_config(1)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    M = np.zeros((db.n, db.m), dtype=np.int64)
    rp = db.row_ptr.astype(np.int64)
    for i in range(db.n):
        M[i, db.col_idx[rp[i]:rp[i + 1]]] = 1
    G = M.T @ M
    rng = np.random.default_rng(0)
    for _ in range(300):
        a, b = rng.integers(0, db.m, size=2)
        assert o.support([min(a, b), max(a, b)] if a != b else [a]) == G[a, b]
    C = pairs.pair_support(db.row_ptr, db.col_idx, db.n, db.m)
    assert (C == G).all()


def test_inclusion_exclusion_identity():
    """|a OR b| = S(a) + S(b) - S(a AND b): OR counted on the dense matrix, AND by the oracle."""
    db = gen.make_config(2, scale=0.05)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    M = pairs.dense_matrix(db.row_ptr, db.col_idx, db.n, db.m, dtype=np.int8).astype(bool)
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = sorted(rng.choice(db.m, size=2, replace=False))
        n_or = int((M[:, a] | M[:, b]).sum())
        assert n_or == o.support([a]) + o.support([b]) - o.support([a, b])


def test_support_matches_horizontal_definition():
    db = gen.make_config(2, scale=0.02)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    T = sets.transactions(db.row_ptr, db.col_idx, db.n, db.m)
    F = o.mine(db.minsup)
    rng = np.random.default_rng(2)
    for idx in rng.choice(len(F), size=min(60, len(F)), replace=False):
        X, v = F[idx]
        assert sets.support(T, X) == v


# ---------------------------------------------------------------- invariants

def test_invariants_on_basket_workload():
    db = gen.make_config(1)
    F, cands = sets.mine(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, count_candidates=True)
    Fd = dict(F)
    # canonical order and shape
    assert [X for X, _ in F] == sorted(X for X, _ in F)
    assert all(all(X[i] < X[i + 1] for i in range(len(X) - 1)) for X, _ in F)
    # anti-monotone support and downward closure
    for X, v in F:
        assert v >= db.minsup
        for i in range(len(X)):
            sub = X[:i] + X[i + 1:]
            if sub:
                assert sub in Fd and Fd[sub] >= v
    # mean support of the frequent sets is at least the threshold (the shape of Table 2)
    assert np.mean([v for _, v in F]) / db.n >= db.minsup / db.n
    # candidate count: sum over prefix classes of q(q-1)/2
    groups = {}
    for X, _ in F:
        groups.setdefault(X[:-1], 0)
        groups[X[:-1]] += 1
    assert cands == sum(q * (q - 1) // 2 for q in groups.values())
    # the C++ oracle agrees on the full workload
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    offs, items, supp, c2 = o.mine_arrays(db.minsup, threads=4)
    assert ocpp.arrays_to_list(offs, items, supp) == F
    assert c2 == cands


def test_paper_table2_direction():
    """Table 2: the mean support of the frequent sets exceeds the threshold at every
    row; the same direction must hold for our oracle at those thresholds."""
    with open(os.path.join(GOLDEN, "paper_tables.json")) as f:
        t = json.load(f)
    for row in t["table2"]:
        assert row["avg_support_pct"] > row["threshold_pct"]
    db = gen.make_config(1)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    prev = None
    for row in t["table2"]:
        s = gen.minsup_from_ppm(row["threshold_pct"] * 10_000, db.n)
        _, _, supp, _ = o.mine_arrays(s)
        mean_pct = 100.0 * supp.mean() / db.n
        assert mean_pct >= row["threshold_pct"]
        if prev is not None:
            assert len(supp) <= prev
        prev = len(supp)


def test_minsup_from_ppm_exact():
    assert gen.minsup_from_ppm(10_000, 10_000) == 100
    assert gen.minsup_from_ppm(2_500, 100_000) == 250
    assert gen.minsup_from_ppm(10_000, 1_000_000) == 10_000
    assert gen.minsup_from_ppm(5_000, 1_000_000) == 5_000
    assert gen.minsup_from_ppm(1, 10) == 1
    for n in range(1, 300):
        for ppm in (1, 999, 5_000, 12_345, 999_999):
            s = gen.minsup_from_ppm(ppm, n)
            # supp >= s  <=>  supp / n >= ppm / 1e6
            assert (s * 1_000_000 >= ppm * n) and ((s - 1) * 1_000_000 < ppm * n or s == 1)


# ---------------------------------------------------------------- certificate

def test_certificate_accepts_exact_result():
    db = gen.make_config(2, scale=0.1)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    F = o.mine_arrays(db.minsup)[:3]
    info = certify.certify(o, F, db.minsup)
    assert info["border_checked"] == info["border_total"]
    info = certify.certify(o, F, db.minsup, pair_closed_form=True, csr=(db.row_ptr, db.col_idx, db.n))
    assert info["border_checked"] == info["border_total"]


def test_certificate_rejects_planted_mistakes():
    db = gen.make_config(1)
    o = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m)
    F = o.mine(db.minsup)
    certify.certify(o, F, db.minsup)
    long_idx = max(range(len(F)), key=lambda i: len(F[i][0]))
    pair_idx = next(i for i, (X, _) in enumerate(F) if len(X) == 2)
    mutants = {
        "dropped maximal set": F[:long_idx] + F[long_idx + 1:],
        "dropped pair": F[:pair_idx] + F[pair_idx + 1:],
        "wrong support": [(X, v + (1 if i == 3 else 0)) for i, (X, v) in enumerate(F)],
        "swapped order": [F[1], F[0]] + F[2:],
        "infrequent extra": sorted(F + [((0, 1, 2, 3, 4, 5), 0)]),
        "duplicate": sorted(F + [F[5]]),
    }
    for name, bad in mutants.items():
        with pytest.raises(certify.CertificateError):
            certify.certify(o, bad, db.minsup)
    # a lower threshold's result is not a certificate for a higher threshold, and v.v.
    F2 = o.mine(db.minsup + 20)
    with pytest.raises(certify.CertificateError):
        certify.certify(o, F2, db.minsup)
    with pytest.raises(certify.CertificateError):
        certify.certify(o, F, db.minsup + 20)


# ---------------------------------------------------------------- generators

def test_generators_deterministic_and_shaped():
    a = gen.make_config(1)
    b = gen.make_config(1)
    assert (a.row_ptr == b.row_ptr).all() and (a.col_idx == b.col_idx).all()
    assert a.n == 10_000 and a.m == 169 and a.minsup == 100
    lens = np.diff(a.row_ptr.astype(np.int64))
    assert 4.0 < lens.mean() < 4.8 and lens.max() <= 32 and lens.min() >= 1
    q = gen.make_config(2, scale=0.1)
    assert q.m == 1000 and q.minsup == 25
    ql = np.diff(q.row_ptr.astype(np.int64))
    assert 8.0 < ql.mean() < 11.0
    for d in (a, q):
        rp = d.row_ptr.astype(np.int64)
        for i in range(0, d.n, max(1, d.n // 50)):
            r = d.col_idx[rp[i]:rp[i + 1]]
            assert (np.diff(r.astype(np.int64)) > 0).all()
    dp = gen.dense_planted(seed=3, n=20_000, m=512, n_patterns=20)
    cs = pairs.column_sums(dp.row_ptr, dp.col_idx, dp.n, dp.m)
    assert cs.max() > 0.08 * dp.n


def test_batch_params_ranges():
    for k in range(256):
        p = gen.batch_params(k)
        assert 1000 <= p["n"] <= 200_000 and 50 <= p["m"] <= 2000
        assert 5 <= p["mean_len"] <= 20 and 5_000 <= p["ppm"] <= 50_000


# ---------------------------------------------------------------- mutation tests

_MUTATIONS = [
    ("skips a later sibling", "cands[idx + 1:]", "cands[idx + 2:]"),
    ("strict threshold", "len(inter) >= minsup", "len(inter) > minsup"),
    ("union instead of intersection", "inter = Tj & T2", "inter = Tj | T2"),
    ("drops first-level threshold", "if len(tid[j]) >= minsup]", "if len(tid[j]) >= 1]"),
    ("reports tidset of sibling", "out.append((X, len(Tj)))", "out.append((X, len(cands[-1][1])))"),
    ("no recursion", "rec(X, nxt)", "pass"),
]


@pytest.mark.parametrize("name,old,new", _MUTATIONS, ids=[m[0] for m in _MUTATIONS])
def test_pins_catch_planted_oracle_mistakes(name, old, new):
    src = open(sets.__file__).read()
    assert old in src, name
    ns = {"__name__": "mutant"}
    exec(compile(src.replace(old, new), "mutant_sets.py", "exec"), ns)
    db, F, _, _ = load_hand_example()
    caught = ns["mine"](db.row_ptr, db.col_idx, db.n, db.m, db.minsup) != F
    for seed in range(6):
        if caught:
            break
        d = gen.random_small(seed, 40, 8, density=0.15 + 0.1 * seed)
        for s in (2, 5, 10):
            if ns["mine"](d.row_ptr, d.col_idx, d.n, d.m, s) != brute.mine(d.row_ptr, d.col_idx, d.n, d.m, s):
                caught = True
                break
    assert caught, f"mutation '{name}' escaped the pins"
