"""Host-only checks of the C-ABI library: it loads, and exports every entry point
that include/bm.h declares.  No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bm.h")
LIB = os.path.join(ROOT, "paper_2412_19420_amd", "libbm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bm_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("bm_build", "bm_pair_support", "bm_mine", "bm_mine_ex", "bm_result_copy",
              "bm_result_info", "bm_result_stats", "bm_db_free", "bm_result_free",
              "bm_item_support", "bm_set_allocator", "bm_last_error", "bm_status_string",
              "bm_abi_version"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\s(bm_[a-z_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbm.so not built")
def test_host_only_entry_points():
    lib = ctypes.CDLL(LIB)
    lib.bm_abi_version.restype = ctypes.c_uint32
    assert lib.bm_abi_version() == 2
    lib.bm_status_string.restype = ctypes.c_char_p
    lib.bm_status_string.argtypes = [ctypes.c_int]
    assert lib.bm_status_string(0) == b"ok"
    assert lib.bm_status_string(2) == b"malformed CSR transaction list"
    lib.bm_result_info.argtypes = [ctypes.c_void_p] * 4
    assert lib.bm_result_info(None, None, None, None) == 1  # BM_ERR_INVALID_ARG
    lib.bm_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.bm_last_error()
    lib.bm_db_free(None)
    lib.bm_result_free(None)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    """The Python binding must refuse to import when libbm.so is absent."""
    import importlib.util
    src = os.path.join(ROOT, "paper_2412_19420_amd", "_bm.py")
    pkg = tmp_path / "fakepkg"
    pkg.mkdir()
    (pkg / "_bm.py").write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("fakepkg._bm", pkg / "_bm.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbm.so not built")
def test_binding_marshalling_checks():
    """Argument marshalling only: element types and contiguity are checked
    before any pointer reaches the library (host tensors suffice here)."""
    import numpy as np
    import torch
    from paper_2412_19420_amd import _bm
    t = torch.arange(10, dtype=torch.int64).to(torch.uint64)
    p, keep = _bm._ptr(t, np.uint64)
    assert p.value == t.data_ptr() and keep is t
    with pytest.raises(TypeError):
        _bm._ptr(t, np.uint32)
    with pytest.raises(ValueError):
        _bm._ptr(torch.zeros((4, 4), dtype=torch.uint32).t(), np.uint32)
    a = np.arange(5, dtype=np.int32)  # converted to the requested element type
    p, keep = _bm._ptr(a, np.uint32)
    assert keep.dtype == np.uint32 and p.value == keep.ctypes.data
    assert _bm._nelem(t) == 10 and _bm._nelem(a) == 5
    assert _bm._ptr(None, np.uint32)[0].value is None


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of bm_options and bm_stats have the header's size and
    field offsets (a C program built with gcc against include/bm.h prints them)."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2412_19420_amd import _bm
    ns = {"BmOptions": _bm.BmOptions, "BmStats": _bm.BmStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bm.h"', 'int main(void) {']
    checks = []
    for cname, pyname in (("bm_options", "BmOptions"), ("bm_stats", "BmStats")):
        cls = ns[pyname]
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        checks.append((f"{cname} size", ctypes.sizeof(cls)))
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
            checks.append((f"{cname} {field}", getattr(cls, field).offset))
    lines += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {" ".join(l.split()[:-1]): int(l.split()[-1]) for l in out.splitlines()}
    for key, want in checks:
        assert got[key] == want, (key, got[key], want)
