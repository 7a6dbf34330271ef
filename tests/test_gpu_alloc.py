"""GPU tests of bm_set_allocator: every device allocation of the library routed
through caller callbacks (here torch's caching allocator), and an allocator
that refuses a request at each point of a build and a mining call in turn --
every such call must fail with BM_ERR_OOM, return every block it had taken,
and leave the library working.  Results are compared with the oracle.

Runs before the other GPU test files (alphabetical order) so that no library
handle of another test is alive when the allocator is switched.
"""
import gc

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
    gc.collect()
    yield bm
    gc.collect()
    bm.bm_set_allocator(None, None)


class TorchAlloc:
    """Device memory from torch's caching allocator; counts live blocks."""

    def __init__(self, fail_at=None):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_at = fail_at  # refuse the request with this 0-based index

    def alloc(self, size, stream):
        i = self.calls
        self.calls += 1
        if self.fail_at is not None and i == self.fail_at:
            return 0
        t = self.torch.empty(size, dtype=self.torch.uint8, device="cuda")
        p = t.data_ptr()
        self.live[p] = t
        return p

    def free(self, ptr, stream):
        self.live.pop(ptr, None)


def _oracle(db, minsup):
    return ocpp.OracleDb(db.row_ptr, db.col_idx, db.n, db.m).mine_arrays(minsup)[:3]


def _same(a, b):
    return all(np.array_equal(np.asarray(x).astype(np.int64), np.asarray(y).astype(np.int64))
               for x, y in zip(a, b))


def _build_and_mine(bm, db, opts=None):
    h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
    try:
        r = bm.bm_mine_ex(h, db.minsup, opts) if opts is not None else bm.bm_mine(h, db.minsup)
        try:
            return r.arrays()
        finally:
            r.free()
    finally:
        h.free()


def test_allocator_routed_to_torch(bm):
    db = gen.make_config(2, scale=0.2)
    want = _oracle(db, db.minsup)
    ta = TorchAlloc()
    gc.collect()
    bm.bm_set_allocator(ta.alloc, ta.free)
    try:
        print("mining with torch's allocator", flush=True)
        got = _build_and_mine(bm, db)
        assert _same(got, want)
        assert ta.calls > 0
        assert not ta.live, f"{len(ta.live)} blocks not returned"
        # subset counting path (long-column routing forced) through the same callbacks
        got = _build_and_mine(bm, db, bm.options(dfs_max_words=1))
        assert _same(got, want)
        assert not ta.live
    finally:
        bm.bm_set_allocator(None, None)
    assert _same(_build_and_mine(bm, db), want)


def test_allocator_refusals_give_oom_and_leak_nothing(bm):
    db = gen.make_config(2, scale=0.05)
    want = _oracle(db, db.minsup)
    probe = TorchAlloc()
    gc.collect()
    bm.bm_set_allocator(probe.alloc, probe.free)
    try:
        _build_and_mine(bm, db)
    finally:
        bm.bm_set_allocator(None, None)
    total = probe.calls
    print(f"{total} allocations in one build + mine", flush=True)
    assert total > 5
    for k in range(total):
        ta = TorchAlloc(fail_at=k)
        bm.bm_set_allocator(ta.alloc, ta.free)
        try:
            with pytest.raises(bm.BmError) as e:
                _build_and_mine(bm, db)
            assert e.value.name == "BM_ERR_OOM", (k, e.value.name)
            gc.collect()
            assert not ta.live, f"refusal {k}: {len(ta.live)} blocks not returned"
        finally:
            bm.bm_set_allocator(None, None)
    # the built-in pool afterwards: still exact
    assert _same(_build_and_mine(bm, db), want)


def test_set_allocator_argument_errors(bm):
    import ctypes
    from paper_2412_19420_amd import _bm
    a = _bm.ALLOC_FN(lambda size, stream, ctx: 0)
    st = _bm.lib.bm_set_allocator(a, _bm.FREE_FN(), None)
    assert st == 1  # BM_ERR_INVALID_ARG: only one of the two callbacks
    # a live handle blocks a switch
    db = gen.from_rows([[0, 1], [1]], m=2)
    h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
    ta = TorchAlloc()
    with pytest.raises(bm.BmError):
        bm.bm_set_allocator(ta.alloc, ta.free)
    h.free()
    bm.bm_set_allocator(ta.alloc, ta.free)
    bm.bm_set_allocator(None, None)
    del ctypes
