"""GPU parity of the association rules (bm_rules_mine) against the rule oracle
(oracle/rules.py) on the oracle's own frequent itemsets: rule lists, supports,
confidence and lift must be identical (conf and lift are quotients of exact
integers below 2^53, so the IEEE doubles agree bit for bit)."""
import numpy as np
import pytest

import gen
from oracle import cpp as ocpp
from oracle import rules as orules

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bm():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.init()
    import paper_2412_19420_amd as bm
    return bm


def _check(bm, db, minsup, ppm, max_len=None):
    h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
    r = bm.bm_mine(h, minsup)
    F = r.to_list()
    F_oracle = ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine(minsup)
    assert F == F_oracle
    want = orules.rules(F_oracle, db.n, ppm, max_len=max_len)
    rs = bm.bm_rules_mine(r, ppm, max_len or 0)
    got = rs.to_list(F)
    assert len(got) == len(want)
    assert got == want
    return got


def test_rules_hand_example(bm):
    from test_oracle import load_hand_example
    from test_oracle_rules import _hand_rules
    db, F, _, _ = load_hand_example()
    want, total0, ppm = _hand_rules()
    got = _check(bm, db, db.minsup, ppm)
    assert [g[:6] for g in got] == want
    assert len(_check(bm, db, db.minsup, 0)) == total0


@pytest.mark.parametrize("seed", range(4))
def test_rules_random_small(bm, seed):
    rng = np.random.default_rng(70 + seed)
    m = int(rng.integers(3, 12))
    n = int(rng.integers(20, 300))
    db = gen.random_small(seed, n, m, density=float(rng.uniform(0.3, 0.7)))
    for ppm in (0, 250_000, 600_000, 1_000_000):
        print(f"rules small seed={seed} n={n} m={m} ppm={ppm}", flush=True)
        _check(bm, db, max(1, n // 6), ppm)


@pytest.mark.parametrize("k,ppm", [(1, 100_000), (1, 700_000), (2, 300_000), (2, 500_000)])
def test_rules_workloads(bm, k, ppm):
    db = gen.make_config(k)
    print(f"rules workload {k} ppm={ppm}", flush=True)
    got = _check(bm, db, db.minsup, ppm)
    assert len(got) > 0


def test_rules_reduced_dense_and_max_len(bm):
    db = gen.make_config(3, scale=0.02)
    print("rules reduced dense", flush=True)
    _check(bm, db, db.minsup, 500_000)
    _check(bm, db, db.minsup, 200_000, max_len=3)


def test_rules_batch_slices_and_errors(bm):
    # rules of each member of a batched result (slices of one store), and the
    # argument errors
    # (members whose itemsets stay short: a frequent set of L items brings at
    # least 3^L - 2^(L+1) + 1 rules with its subsets, which the pure-Python oracle
    # could not list for the 18-item sets of member 1)
    dbs = [gen.batch_db(k, scale=0.05) for k in (0, 2, 4, 6, 7)]
    hs = [bm.bm_build(d.row_ptr, d.col_idx, d.n, d.m) for d in dbs]
    rs = bm.bm_mine_batch(hs, [d.minsup for d in dbs])
    for d, r in zip(dbs, rs):
        print(f"rules of batch member {d.name}", flush=True)
        F = r.to_list()
        want = orules.rules(F, d.n, 400_000)
        assert bm.bm_rules_mine(r, 400_000).to_list(F) == want
    with pytest.raises(bm.BmError) as e:
        bm.bm_rules_mine(rs[0], 1_000_001)
    assert e.value.name == "BM_ERR_INVALID_ARG"
    with pytest.raises(bm.BmError) as e:
        bm.bm_rules_mine(rs[0], 0, max_len=25)
    assert e.value.name == "BM_ERR_UNSUPPORTED"
    empty = bm.bm_mine(hs[0], dbs[0].n + 1)
    assert len(bm.bm_rules_mine(empty, 0)) == 0
