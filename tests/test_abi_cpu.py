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


def test_ctypes_layouts_match_the_header(tmp_path):
    """Compile a C probe against include/irgl.h and compare sizes/offsets with
    the binding's ctypes structures."""
    import subprocess
    from paper_1607_05707_amd import irgl
    structs = {"irgl_csr": irgl.irgl_csr, "irgl_config": irgl.irgl_config, "irgl_stats": irgl.irgl_stats,
               "irgl_mst_config": irgl.irgl_mst_config,
               "irgl_task": irgl.irgl_task, "irgl_batch_config": irgl.irgl_batch_config,
               "irgl_mesh": irgl.irgl_mesh, "irgl_dmr_config": irgl.irgl_dmr_config,
               "irgl_dmr_stats": irgl.irgl_dmr_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "irgl.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for name, cls in structs.items():
        assert int(got[f"{name} size"]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_control_block_sizes_is_the_intersection():
    from paper_1607_05707_amd import irgl
    assert irgl.irgl_control_block_sizes() == [256, 512, 1024]


def test_batch_argument_errors_without_device():
    from paper_1607_05707_amd import irgl
    L = irgl._lib
    out = ctypes.c_size_t()
    assert L.irgl_batch_workspace_bytes(None, 3, None, ctypes.byref(out)) == irgl.IRGL_ERR_INVALID_ARGUMENT
    arr = (irgl.irgl_task * 1)()
    assert L.irgl_batch_workspace_bytes(arr, 1, None, ctypes.byref(out)) == irgl.IRGL_ERR_INVALID_ARGUMENT
    h = ctypes.c_void_p()
    assert L.irgl_batch_submit(arr, 0, 0x1000, 100, None, None, ctypes.byref(h)) == irgl.IRGL_ERR_INVALID_ARGUMENT
    assert L.irgl_batch_wait(None, None) == irgl.IRGL_ERR_INVALID_ARGUMENT
    assert L.irgl_batch_free(None) == irgl.IRGL_OK


def test_dmr_argument_errors_without_device():
    from paper_1607_05707_amd import irgl
    L = irgl._lib
    INV = irgl.IRGL_ERR_INVALID_ARGUMENT
    out = ctypes.c_size_t()
    assert L.irgl_dmr_workspace_bytes(None, ctypes.byref(out)) == INV
    m = irgl.irgl_mesh()
    m.pts, m.tri, m.nbr = 0x1000, 0x2000, 0x3000
    for npts, ntri, pcap, tcap in [(2, 1, 10, 10), (3, 0, 10, 10), (5, 1, 4, 10), (5, 4, 10, 3),
                                   (5, 4, 10, 1 << 30)]:
        m.npts, m.ntri, m.pcap, m.tcap = npts, ntri, pcap, tcap
        assert L.irgl_dmr_workspace_bytes(ctypes.byref(m), ctypes.byref(out)) == INV, (npts, ntri, pcap, tcap)
    m.npts, m.ntri, m.pcap, m.tcap = 4, 2, 16, 16
    assert L.irgl_dmr_workspace_bytes(ctypes.byref(m), ctypes.byref(out)) == irgl.IRGL_OK
    assert L.irgl_dmr_refine(ctypes.byref(m), None, 0, None, None, None) == INV
    assert L.irgl_dmr_refine(ctypes.byref(m), 0x4000, out.value - 1, None, None, None) == \
        irgl.IRGL_ERR_WORKSPACE_TOO_SMALL
    cfg = irgl.irgl_dmr_config()
    for field, value in (("min_angle", 60.0), ("block", 512)):
        cfg = irgl.irgl_dmr_config()
        setattr(cfg, field, value)
        assert L.irgl_dmr_refine(ctypes.byref(m), 0x4000, out.value, ctypes.byref(cfg), None, None) == \
            irgl.IRGL_ERR_CONFIG, field
