"""Pins of the association-rule oracle (oracle/rules.py) -- CPU only.

The oracle is fixed by things other than itself: rules derived by hand for the
hand-worked example; a brute force that enumerates every pair of disjoint
non-empty itemsets over the raw transactions (horizontal subset tests, no use
of the mined list); the closed-form rule count at threshold 0; symmetry of
lift; and planted mistakes, each of which must fail one of these pins.
"""
import os
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import gen
from oracle import brute, rules

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _hand_rules():
    out, total0, ppm = [], None, None
    with open(os.path.join(GOLDEN, "hand_rules.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "min_conf_ppm":
                ppm = int(tok[1])
            elif tok[0] == "TOTAL0":
                total0 = int(tok[1])
            elif tok[0] == "R":
                a = tok.index("=>")
                c = tok.index(":")
                out.append((int(tok[1]), tuple(int(x) for x in tok[2:a]),
                            tuple(int(x) for x in tok[a + 1:c]), int(tok[c + 1]), int(tok[c + 2]),
                            int(tok[c + 3])))
    return out, total0, ppm


def _hand_db():
    from test_oracle import load_hand_example
    db, F, _, _ = load_hand_example()
    return db, F


def _check_hand(rules_fn):
    db, F = _hand_db()
    want, total0, ppm = _hand_rules()
    got = rules_fn(F, db.n, ppm)
    assert [r[:6] for r in got] == want
    for zi, X, Y, sx, sy, sz, conf, lift in got:
        assert abs(Fraction(conf) - Fraction(sz, sx)) <= Fraction(1, 2 ** 50)
        assert abs(Fraction(lift) - Fraction(sz * db.n, sx * sy)) <= Fraction(1, 2 ** 48)
    assert len(rules_fn(F, db.n, 0)) == total0


def test_hand_example_rules():
    _check_hand(rules.rules)


def _brute_rules(db, minsup, ppm):
    """Every (X, Y) disjoint, non-empty, over the items, with supports counted
    from the transactions directly; kept when X + Y is frequent and the
    confidence passes."""
    rows = [set(db.col_idx[db.row_ptr[i]:db.row_ptr[i + 1]].tolist()) for i in range(db.n)]

    def supp(s):
        return sum(1 for r in rows if s <= r)

    F = brute.mine(db.row_ptr, db.col_idx, db.n, db.m, minsup)
    index = {x: i for i, (x, _) in enumerate(F)}
    out = []
    items = list(range(db.m))
    for kz in range(2, db.m + 1):
        for Z in combinations(items, kz):
            sz = supp(set(Z))
            if sz < minsup:
                continue
            for kx in range(1, kz):
                for X in combinations(Z, kx):
                    Y = tuple(z for z in Z if z not in X)
                    sx, sy = supp(set(X)), supp(set(Y))
                    if Fraction(sz, sx) >= Fraction(ppm, 10 ** 6):
                        out.append((index[Z], X, Y, sx, sy, sz))
    out.sort(key=lambda r: (r[0], r[1]))
    return F, out


@pytest.mark.parametrize("seed", range(6))
def test_rules_match_brute_force(seed):
    rng = np.random.default_rng(50 + seed)
    m = int(rng.integers(2, 8))
    n = int(rng.integers(5, 60))
    db = gen.random_small(seed, n, m, density=float(rng.uniform(0.3, 0.7)))
    minsup = max(1, n // 5)
    for ppm in (0, 300_000, 500_000, 800_000, 1_000_000):
        F, want = _brute_rules(db, minsup, ppm)
        got = rules.rules(F, db.n, ppm)
        assert [r[:6] for r in got] == want, (seed, ppm)


def test_rule_invariants():
    db = gen.make_config(1)
    from oracle import sets
    F = sets.mine(db.row_ptr, db.col_idx, db.n, db.m, db.minsup)
    all_rules = rules.rules(F, db.n, 0)
    assert len(all_rules) == sum(2 ** len(x) - 2 for x, _ in F if len(x) >= 2)
    lift = {(r[1], r[2]): r[7] for r in all_rules}
    for (X, Y), v in lift.items():
        assert lift[(Y, X)] == v  # lift is symmetric in X and Y
    for r in all_rules:
        assert 0 < r[6] <= 1.0
    # max_len drops exactly the rules of longer sets
    short = rules.rules(F, db.n, 0, max_len=2)
    assert len(short) == sum(2 for x, _ in F if len(x) == 2)


_MUTATIONS = [
    ("confidence over the consequent", "float(sz) / float(sx)", "float(sz) / float(sy)"),
    ("lift without n", "float(int(sz) * int(n))", "float(int(sz))"),
    ("strict threshold", ">= int(min_conf_ppm) * sx", "> int(min_conf_ppm) * sx"),
    ("consequent may be empty", "for k in range(1, L):", "for k in range(1, L + 1):"),
    ("ordered by consequent", "out.sort(key=lambda r: (r[0], r[1]))",
     "out.sort(key=lambda r: (r[0], r[2]))"),
]


@pytest.mark.parametrize("name,old,new", _MUTATIONS, ids=[m[0] for m in _MUTATIONS])
def test_pins_catch_planted_rule_mistakes(name, old, new):
    src = open(rules.__file__).read()
    assert old in src, name
    ns = {"__name__": "mutant"}
    exec(compile(src.replace(old, new), "mutant_rules.py", "exec"), ns)
    try:
        _check_hand(ns["rules"])
    except (AssertionError, KeyError):
        return
    pytest.fail(f"mutation '{name}' escaped the pins")
