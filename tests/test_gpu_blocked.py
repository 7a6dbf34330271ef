"""GPU parity of out-of-core mining (bm_mine_blocked): the transactions stay in
host memory and the device holds one row block at a time; supports are summed
over the blocks.  The result must equal the oracle's arrays (and bm_mine's)
for every block size: one block, many blocks, blocks that are not a whole
number of 64-bit words, a ragged last block, and wide databases that take the
atomic pack.  Also the Table 1/2-style sweep's own oracle check."""
import numpy as np
import pytest

import gen
from oracle import cpp as ocpp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bm():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.init()
    import paper_2412_19420_amd as bm
    return bm


def _oracle(db, minsup):
    return ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine_arrays(minsup)


def _same(a, b):
    return all(np.array_equal(np.asarray(x).astype(np.int64), np.asarray(y).astype(np.int64))
               for x, y in zip(a, b))


@pytest.mark.parametrize("k,scale,blocks", [
    (1, 1.0, [10_000, 4096, 1000, 777, 64]),
    (2, 1.0, [100_000, 25_000, 30_001]),
    (3, 0.05, [50_000, 12_288, 10_000]),
    (5, 0.02, [20_000, 4_999]),
])
def test_blocked_equals_oracle(bm, k, scale, blocks):
    db = gen.make_config(k, scale=scale)
    want = _oracle(db, db.minsup)
    for R in blocks:
        print(f"blocked workload {k} scale {scale}: n={db.n} block_rows={R}", flush=True)
        r = bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, R)
        assert _same(r.arrays(), want[:3]), R
        assert r.stats()["candidates_total"] == want[3]


def test_blocked_wide_and_degenerate(bm):
    # more items than the tiled pack takes (atomic pack per block), empty rows,
    # duplicates; an empty database; minsup above n
    rng = np.random.default_rng(21)
    n, m = 2_500, 20_000
    lens = rng.poisson(30, n)
    lens[rng.random(n) < 0.05] = 0
    rp = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=rp[1:])
    ci = (rng.zipf(1.3, int(rp[-1])) % m).astype(np.uint32)
    db = gen.Db("wide", rp, ci, n, m, 25)
    want = _oracle(db, 25)
    for R in (2_500, 1_000, 333):
        print(f"blocked wide block_rows={R}", flush=True)
        assert _same(bm.bm_mine_blocked(rp, ci, n, m, 25, R).arrays(), want[:3])
    e = gen.from_rows([], m=4)
    assert len(bm.bm_mine_blocked(e.row_ptr, e.col_idx, 0, 4, 1, 16)) == 0
    small = gen.make_config(1)
    assert len(bm.bm_mine_blocked(small.row_ptr, small.col_idx, small.n, small.m,
                                  small.n + 1, 1000)) == 0


def test_blocked_errors(bm):
    import torch
    db = gen.make_config(1)
    with pytest.raises(bm.BmError) as e:
        bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, 0)
    assert e.value.name == "BM_ERR_INVALID_ARG"
    with pytest.raises(bm.BmError) as e:
        bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, 0, 1000)
    assert e.value.name == "BM_ERR_INVALID_ARG"
    bad = db.col_idx.copy()
    bad[len(bad) - 3] = db.m
    with pytest.raises(bm.BmError) as e:
        bm.bm_mine_blocked(db.row_ptr, bad, db.n, db.m, db.minsup, 1000)
    assert e.value.name == "BM_ERR_CSR"
    rp = db.row_ptr.copy()
    rp[4321] = rp[4323] + 1  # decreasing inside the fifth block
    with pytest.raises(bm.BmError) as e:
        bm.bm_mine_blocked(rp, db.col_idx, db.n, db.m, db.minsup, 1000)
    assert e.value.name == "BM_ERR_CSR"
    # device memory is refused: the point is a database that stays on the host
    from paper_2412_19420_amd import _bm
    import ctypes
    drp = torch.from_numpy(db.row_ptr.astype(np.uint64)).cuda()
    dci = torch.from_numpy(db.col_idx.astype(np.uint32)).cuda()
    h = ctypes.c_void_p()
    st = _bm.lib.bm_mine_blocked(ctypes.c_void_p(drp.data_ptr()), ctypes.c_void_p(dci.data_ptr()),
                                 db.n, db.m, db.minsup, 1000, None, None, ctypes.byref(h))
    assert st == 1  # BM_ERR_INVALID_ARG
    # the library still works
    assert _same(bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, 1000).arrays(),
                 _oracle(db, db.minsup)[:3])


def test_blocked_full_dense_planted(bm):
    # the 1M x 4,096 dense workload in four row blocks, against the oracle's
    # complete result stored in tests/golden
    from test_gpu_mine import _load_full_fixture
    db = gen.make_config(3)
    want, cands, _ = _load_full_fixture("full_dense_planted_1M.npz")
    print("blocked dense 1M in 4 blocks", flush=True)
    r = bm.bm_mine_blocked(db.row_ptr, db.col_idx, db.n, db.m, db.minsup, 250_000)
    assert _same(r.arrays(), want)
    assert r.stats()["candidates_total"] == cands


def test_table_sweep_points_equal_oracle(bm):
    import torch
    import bench
    out = bench.table_sweep(bm, torch, reps=1)
    assert len(out["points"]) == 25
    assert all(p["equals_oracle"] for p in out["points"])
    # Table 2's direction: the mean support of the frequent sets is at least the threshold
    for p in out["points"]:
        if p["frequent_itemsets"]:
            assert p["avg_support_pct"] >= p["threshold_pct"] - 1e-9
        assert p["peak_device_mb"] is not None and p["peak_device_mb"] > 0
