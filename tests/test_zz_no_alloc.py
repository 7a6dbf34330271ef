"""GPU test of the allocation-free pair-support entry point
(bm_pair_support_noalloc): through the C ABI, its output must equal
bm_pair_support's (and the Gram closed form) on two calls in a row, the second
with a smaller input, and it must request no device memory: with every library
allocation routed through a counting allocator, the count does not move
during the call."""
import ctypes
import gc

import numpy as np
import pytest

import gen
from oracle import pairs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bm():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.init()
    import paper_2412_19420_amd as bm
    return bm


def _noalloc(bm, db_handle, items_t, k, out_t):
    from paper_2412_19420_amd import _bm
    st = _bm.lib.bm_pair_support_noalloc(
        db_handle.handle, ctypes.c_void_p(items_t.data_ptr() if items_t is not None else 0),
        ctypes.c_uint32(k), ctypes.c_void_p(out_t.data_ptr()),
        ctypes.c_void_p(__import__("torch").cuda.current_stream().cuda_stream))
    return st


def _setup_lib(bm):
    from paper_2412_19420_amd import _bm
    _bm.lib.bm_pair_support_noalloc.restype = ctypes.c_int
    _bm.lib.bm_pair_support_noalloc.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_uint32] + \
        [ctypes.c_void_p] * 2
    return _bm


@pytest.mark.parametrize("first,second", [((4000, 300, 0.1, 300), (1500, 90, 0.2, 70)),
                                          ((70_001, 600, 0.05, 512), (2000, 40, 0.3, 9))])
def test_noalloc_matches_pair_support_twice(bm, first, second):
    import torch
    _bm = _setup_lib(bm)
    for n, m, density, k in (first, second):
        print(f"noalloc pair support n={n} m={m} k={k}", flush=True)
        rng = np.random.default_rng(n + m + k)
        rows = [list(np.nonzero(rng.random(m) < density)[0]) for _ in range(n)]
        db = gen.from_rows(rows, m=m)
        h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
        items = rng.integers(0, m, size=k).astype(np.uint32)
        items[k // 2] = items[0]
        ref = bm.bm_pair_support(h, items)
        dit = torch.from_numpy(items).cuda()
        out = torch.full((k * k,), 0xFFFFFFFF, dtype=torch.uint32, device="cuda")
        assert _noalloc(bm, h, dit, k, out) == 0, _bm.lib.bm_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(k, k)
        assert np.array_equal(got, np.asarray(ref).reshape(k, k))
        want = pairs.pair_support(db.row_ptr, db.col_idx, db.n, db.m, cols=items)
        assert np.array_equal(got.astype(np.int64), np.asarray(want).astype(np.int64))
        # items == NULL: every item in id order
        out2 = torch.zeros(m * m, dtype=torch.uint32, device="cuda")
        assert _noalloc(bm, h, None, m, out2) == 0, _bm.lib.bm_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy().reshape(m, m), np.asarray(bm.bm_pair_support(h)))


def test_noalloc_makes_no_allocation_and_rejects_bad_arguments(bm):
    import torch
    _bm = _setup_lib(bm)
    calls = [0]
    live = {}

    def alloc(size, stream):
        calls[0] += 1
        t = torch.empty(size, dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, stream):
        live.pop(ptr, None)

    db = gen.make_config(2, scale=0.1)
    k = 200
    items = torch.from_numpy(np.arange(k, dtype=np.uint32)).cuda()
    out = torch.zeros(k * k, dtype=torch.uint32, device="cuda")
    gc.collect()
    bm.bm_set_allocator(alloc, free)
    try:
        h = bm.bm_build(db.row_ptr, db.col_idx, db.n, db.m)
        before = calls[0]
        assert _noalloc(bm, h, items, k, out) == 0, _bm.lib.bm_last_error()
        torch.cuda.synchronize()
        assert calls[0] == before, "the allocation-free call requested device memory"
        ref = bm.bm_pair_support(h, items.cpu().numpy())  # allocates: the reference call
        assert np.array_equal(out.cpu().numpy().reshape(k, k), np.asarray(ref))
        before = calls[0]
        # errors: too many items, host output, host items
        big = torch.from_numpy(np.zeros(2049, dtype=np.uint32)).cuda()
        assert _noalloc(bm, h, big, 2049, out) == 5  # BM_ERR_UNSUPPORTED
        host_out = np.zeros(k * k, dtype=np.uint32)
        st = _bm.lib.bm_pair_support_noalloc(h.handle, ctypes.c_void_p(items.data_ptr()), k,
                                             host_out.ctypes.data_as(ctypes.c_void_p), None)
        assert st == 1  # BM_ERR_INVALID_ARG
        host_items = np.arange(k, dtype=np.uint32)
        st = _bm.lib.bm_pair_support_noalloc(h.handle, host_items.ctypes.data_as(ctypes.c_void_p),
                                             k, ctypes.c_void_p(out.data_ptr()), None)
        assert st == 1
        bad_h = np.arange(k, dtype=np.uint32)
        bad_h[3] = db.m
        bad = torch.from_numpy(bad_h).cuda()
        assert _noalloc(bm, h, bad, k, out) == 1  # an item id >= n_items
        assert calls[0] == before
        h.free()
    finally:
        gc.collect()
        bm.bm_set_allocator(None, None)
