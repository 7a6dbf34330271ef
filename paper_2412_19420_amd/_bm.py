"""ctypes binding of libbm.so: argument marshalling only.

Every computation runs in the HIP library; this module converts Python/numpy/
torch arguments to pointers and sizes and wraps the opaque handles.  It raises
ImportError when the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python paper_2412_19420_amd/build.py or __graft_entry__.build())")

# When PyTorch-ROCm is installed, its HIP runtime is loaded before the library
# so that the library binds to that same runtime: the two then share one device
# context, and torch streams and tensors can be passed across the boundary.
try:
    import torch as _torch
except ImportError:
    _torch = None

lib = ctypes.CDLL(LIB_PATH)

BM_MAX_LEVELS = 64
BM_K_NAMES = ["build", "colsum", "gram_mfma", "andpop", "andpop_reg", "level", "emit", "dfs",
              "sched", "gram_mfma_big", "gram_small", "project"]
BM_K_COUNT = len(BM_K_NAMES)

FLAG_TIMING = 1
FLAG_NO_MFMA = 2
FLAG_ALL_MFMA = 4
FLAG_GRAPH = 8
FLAG_TRACE = 16
FLAG_SHUFFLE = 32
FLAG_LEVELSYNC = 64
FLAG_FP4_MFMA = 128
FLAG_INT8_MFMA = 256
FLAG_DFS_BLOCK_ONLY = 512
FLAG_TIMING_MAIN = 1024
FLAG_DEPTH_FIRST = 2048
FLAG_NO_PROJECT = 4096
MLP_PARAMS = 4801

STATUS = {0: "BM_OK", 1: "BM_ERR_INVALID_ARG", 2: "BM_ERR_CSR", 3: "BM_ERR_OOM",
          4: "BM_ERR_DEVICE", 5: "BM_ERR_UNSUPPORTED"}


class BmStats(ctypes.Structure):
    _fields_ = [
        ("max_len", ctypes.c_uint32),
        ("n_frequent_items", ctypes.c_uint32),
        ("candidates", ctypes.c_uint64 * (BM_MAX_LEVELS + 1)),
        ("frequent", ctypes.c_uint64 * (BM_MAX_LEVELS + 1)),
        ("candidates_total", ctypes.c_uint64),
        ("frequent_total", ctypes.c_uint64),
        ("classes_mfma", ctypes.c_uint64),
        ("classes_andpop", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double * BM_K_COUNT),
        ("kernel_launches", ctypes.c_uint64 * BM_K_COUNT),
        ("kernel_bytes", ctypes.c_double * BM_K_COUNT),
        ("kernel_ops", ctypes.c_double * BM_K_COUNT),
        ("wall_ms", ctypes.c_double),
        ("host_syncs", ctypes.c_uint32),
        ("dfs_tasks", ctypes.c_uint64),
        ("mfma_form", ctypes.c_uint32),
    ]


class BmOptions(ctypes.Structure):
    _fields_ = [
        ("flags", ctypes.c_uint32),
        ("mfma_min_children", ctypes.c_uint32),
        ("andpop_chunk_words", ctypes.c_uint32),
        ("split_words", ctypes.c_uint32),
        ("shuffle_seed", ctypes.c_uint32),
        ("dfs_threads", ctypes.c_uint32),
        ("dfs_max_words", ctypes.c_uint32),
        ("mfma_big_children", ctypes.c_uint32),
        ("dfs_wave_max_words", ctypes.c_uint32),
        ("subset_max_children", ctypes.c_uint32),
        ("dfs_arena_nodes", ctypes.c_uint32),
        ("project_gain", ctypes.c_uint32),
    ]


_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)

lib.bm_abi_version.restype = ctypes.c_uint32
lib.bm_status_string.restype = ctypes.c_char_p
lib.bm_status_string.argtypes = [ctypes.c_int]
lib.bm_last_error.restype = ctypes.c_char_p
lib.bm_release_cached_memory.restype = ctypes.c_int
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
lib.bm_set_allocator.restype = ctypes.c_int
lib.bm_set_allocator.argtypes = [ALLOC_FN, FREE_FN, ctypes.c_void_p]
lib.bm_build.restype = ctypes.c_int
lib.bm_build.argtypes = [_vp, _vp, ctypes.c_uint64, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
lib.bm_db_info.restype = ctypes.c_int
lib.bm_db_info.argtypes = [_vp, _u64p, _u32p, _u64p]
lib.bm_item_support.restype = ctypes.c_int
lib.bm_item_support.argtypes = [_vp, _vp, _vp]
lib.bm_pair_support.restype = ctypes.c_int
lib.bm_pair_support.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp]
lib.bm_mine.restype = ctypes.c_int
lib.bm_mine.argtypes = [_vp, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
lib.bm_mine_ex.restype = ctypes.c_int
lib.bm_mine_ex.argtypes = [_vp, ctypes.c_uint32, ctypes.POINTER(BmOptions), _vp, ctypes.POINTER(_vp)]
lib.bm_mine_blocked.restype = ctypes.c_int
lib.bm_mine_blocked.argtypes = [_vp, _vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.POINTER(BmOptions), _vp, ctypes.POINTER(_vp)]
lib.bm_mine_batch.restype = ctypes.c_int
lib.bm_mine_batch.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                              _vp, ctypes.POINTER(BmOptions), _vp, ctypes.POINTER(_vp)]
lib.bm_result_info.restype = ctypes.c_int
lib.bm_result_info.argtypes = [_vp, _u64p, _u64p, _u32p]
lib.bm_result_copy.restype = ctypes.c_int
lib.bm_result_copy.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.bm_result_stats.restype = ctypes.c_int
lib.bm_result_stats.argtypes = [_vp, ctypes.POINTER(BmStats)]
_f32p = ctypes.POINTER(ctypes.c_float)
lib.bm_result_trace.restype = ctypes.c_int
lib.bm_result_trace.argtypes = [_vp, _vp, _vp, _u64p]
lib.bm_model_create.restype = ctypes.c_int
lib.bm_model_create.argtypes = [ctypes.c_uint32, ctypes.POINTER(_vp)]
lib.bm_model_load.restype = ctypes.c_int
lib.bm_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_vp)]
lib.bm_model_save.restype = ctypes.c_int
lib.bm_model_save.argtypes = [_vp, ctypes.c_char_p]
lib.bm_model_train.restype = ctypes.c_int
lib.bm_model_train.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float,
                               ctypes.c_uint32, _f32p, _vp]
lib.bm_model_train_ex.restype = ctypes.c_int
lib.bm_model_train_ex.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float,
                                  ctypes.c_uint32, ctypes.c_uint32, _f32p, _vp]
lib.bm_model_predict.restype = ctypes.c_int
lib.bm_model_predict.argtypes = [_vp, _vp, ctypes.c_uint64, _vp, _vp]
lib.bm_model_grad.restype = ctypes.c_int
lib.bm_model_grad.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, _vp, _f32p, _vp]
lib.bm_model_params.restype = ctypes.c_int
lib.bm_model_params.argtypes = [_vp, _vp, _vp, _vp]
lib.bm_model_set_params.restype = ctypes.c_int
lib.bm_model_set_params.argtypes = [_vp, _vp, _vp]
lib.bm_build_batch.restype = ctypes.c_int
lib.bm_build_batch.argtypes = [ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp]
lib.bm_autotune.restype = ctypes.c_int
lib.bm_autotune.argtypes = [_vp, _vp, ctypes.c_uint32, _vp, _vp, ctypes.c_uint32, _vp, _vp,
                            ctypes.POINTER(ctypes.c_double)]
lib.bm_model_free.restype = None
lib.bm_model_free.argtypes = [_vp]
lib.bm_db_free.restype = None
lib.bm_db_free.argtypes = [_vp]
lib.bm_result_free.restype = None
lib.bm_result_free.argtypes = [_vp]
lib.bm_rules_mine.restype = ctypes.c_int
lib.bm_rules_mine.argtypes = [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
lib.bm_rules_info.restype = ctypes.c_int
lib.bm_rules_info.argtypes = [_vp, _u64p]
lib.bm_rules_copy.restype = ctypes.c_int
lib.bm_rules_copy.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
lib.bm_rules_free.restype = None
lib.bm_rules_free.argtypes = [_vp]


class BmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        detail = lib.bm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {self.name}: {detail}")


def check(status: int, where: str):
    if status != 0:
        raise BmError(status, where)


def _stream_ptr(stream):
    """hipStream_t of `stream` (torch.cuda.Stream, int handle, or None = torch's current stream)."""
    if stream is None:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


_TORCH_DTYPE = ({np.uint64: _torch.uint64, np.uint32: _torch.uint32, np.int64: _torch.int64}
                if _torch is not None else {})


def _nelem(a) -> int:
    """Element count of a numpy array or torch tensor (numel: len() of a tensor is slow)."""
    if _torch is not None and isinstance(a, _torch.Tensor):
        return a.numel()
    return len(a)


def _ptr(a, dtype):
    """(pointer, keepalive) of a numpy array or torch tensor with the given element dtype."""
    if a is None:
        return ctypes.c_void_p(0), None
    if _torch is not None and isinstance(a, _torch.Tensor):
        want = _TORCH_DTYPE[dtype]
        if a.dtype != want:
            raise TypeError(f"tensor dtype {a.dtype}, expected {want}")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), arr
