"""C-ABI checks that need no GPU: the library loads, exports every function
include/irgl.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1607_05707_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irgl.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irgl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_build.LIB):
        pytest.fail("libirgl.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(_build.LIB)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("irgl_graph_upload", "irgl_graph_free", "irgl_workspace_bytes", "irgl_bfs",
                     "irgl_sssp", "irgl_query_status", "irgl_status_string", "irgl_version"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_names_match_abi():
    from paper_1607_05707_amd import irgl
    missing = [n for n in _declared_functions() if not hasattr(irgl, n)]
    assert not missing, f"binding lacks: {missing}"


def test_version_and_status_strings(lib):
    lib.irgl_version.restype = ctypes.c_int
    assert lib.irgl_version() == 100
    lib.irgl_status_string.restype = ctypes.c_char_p
    seen = set()
    for code in range(15):
        s = lib.irgl_status_string(code).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 15
    assert lib.irgl_status_string(999).decode() == "unknown status"


def test_argument_errors_without_device():
    from paper_1607_05707_amd import irgl
    L = irgl._lib
    INV = irgl.IRGL_ERR_INVALID_ARGUMENT
    h = ctypes.c_void_p()
    assert L.irgl_graph_upload(None, ctypes.byref(h)) == INV
    csr = irgl.irgl_csr()
    assert L.irgl_graph_upload(ctypes.byref(csr), None) == INV
    fake = 0x1000
    for n, m, rp, col in [(0, 0, fake, fake), (-5, 0, fake, fake), (10, -1, fake, fake),
                          (10, 1 << 31, fake, fake), (10, 5, None, fake), (10, 5, fake, None)]:
        csr.n, csr.m, csr.row_ptr, csr.col, csr.w, csr.flags = n, m, rp, col, None, 0
        assert L.irgl_graph_upload(ctypes.byref(csr), ctypes.byref(h)) == INV, (n, m, rp, col)
    out = ctypes.c_size_t()
    assert L.irgl_workspace_bytes(None, 0, 0, None, ctypes.byref(out)) == INV
    assert L.irgl_bfs(None, 0, fake, None, fake, 1 << 20, None, None, None) == INV
    assert L.irgl_sssp(None, 0, fake, None, fake, 1 << 20, None, None, None) == INV
    st = irgl.irgl_stats()
    assert L.irgl_query_status(None, None, ctypes.byref(st)) == INV
    assert L.irgl_graph_free(None) == irgl.IRGL_OK


def test_no_device_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1607_05707_amd import irgl
    csr = irgl.irgl_csr()
    csr.n, csr.m, csr.row_ptr, csr.col, csr.w, csr.flags = 10, 5, 0x1000, 0x2000, None, 0
    h = ctypes.c_void_p()
    assert irgl._lib.irgl_graph_upload(ctypes.byref(csr), ctypes.byref(h)) == irgl.IRGL_ERR_NO_DEVICE
    assert h.value is None
