"""Python binding of the C ABI in ``include/irgl.h`` (argument marshalling only).

Every function named ``irgl_*`` here calls the C entry point of the same name
in ``_lib/libirgl.so``; all graph work runs in that library's HIP kernels.
Device memory and streams come from PyTorch: graph arrays, outputs and
workspaces are CUDA (HIP) tensors, streams are ``torch.cuda.Stream`` objects.

Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libirgl.so")

INF = 0xFFFFFFFF

IRGL_OK = 0
IRGL_ERR_INVALID_ARGUMENT = 1
IRGL_ERR_NO_WEIGHTS = 2
IRGL_ERR_INVALID_GRAPH = 3
IRGL_ERR_WORKSPACE_TOO_SMALL = 4
IRGL_ERR_OVERFLOW = 5
IRGL_ERR_ABORTED = 6
IRGL_ERR_BUSY = 7
IRGL_ERR_TOO_LARGE = 8
IRGL_ERR_NO_DEVICE = 9
IRGL_ERR_DEVICE = 10
IRGL_ERR_WATCHDOG = 11
IRGL_ERR_ITERATION_LIMIT = 12
IRGL_ERR_CONFIG = 13
IRGL_ERR_INTERNAL = 14

IRGL_KIND_BFS = 0
IRGL_KIND_SSSP = 1
IRGL_SYMMETRIC = 1
IRGL_VALIDATE = 2
IRGL_MODE_PERSISTENT = 0
IRGL_MODE_HOST_LOOP = 1
IRGL_MODE_TOPOLOGY = 2
IRGL_REDUCE_ANY = 0
IRGL_REDUCE_ALL = 1
IRGL_WATCHDOG_IMMEDIATE = 0xFFFFFFFF
IRGL_BITMAP_NEVER = 0xFFFFFFFF
IRGL_GRID_TIER_OFF = -1
IRGL_DELTA_NONE = 0xFFFFFFFF
IRGL_DO_OFF = 0xFFFFFFFF
IRGL_BARRIER_XCD = 0
IRGL_BARRIER_WORKGROUP = 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build() or python -m paper_1607_05707_amd._build)")
_lib = ctypes.CDLL(LIB_PATH)


class irgl_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class irgl_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("t_wave", ctypes.c_int32), ("t_block", ctypes.c_int32),
                ("t_grid", ctypes.c_int32), ("grid", ctypes.c_int32), ("mode", ctypes.c_int32), ("max_iter", ctypes.c_uint32),
                ("wl_capacity", ctypes.c_uint32), ("watchdog_ms", ctypes.c_uint32),
                ("abort_flag", ctypes.c_void_p), ("t_bitmap", ctypes.c_uint32),
                ("trace_len", ctypes.c_uint32), ("do_alpha", ctypes.c_uint32), ("do_beta", ctypes.c_uint32),
                ("delta", ctypes.c_uint32), ("trace", ctypes.c_void_p), ("barrier", ctypes.c_uint32),
                ("reduce", ctypes.c_uint32)]


class irgl_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_uint32),
                ("items", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("max_frontier", ctypes.c_uint32), ("grid", ctypes.c_int32),
                ("block", ctypes.c_int32), ("heavy_pulls", ctypes.c_uint32),
                ("frontier_edges", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


STATS_BYTES = ctypes.sizeof(irgl_stats)

_c = ctypes.c_void_p
_lib.irgl_version.restype = ctypes.c_int
_lib.irgl_version.argtypes = []
_lib.irgl_shutdown.restype = ctypes.c_int32
_lib.irgl_shutdown.argtypes = []

# Every live graph, batch and server handle.  At interpreter exit they are
# released (servers closed, batches and graphs freed) and the library's
# pinned words returned with irgl_shutdown(), all while the HIP runtime is
# still up; finalizers that run later find their handles already released.
_live = weakref.WeakSet()
_shut = False


def _release_all() -> None:
    global _shut
    if _shut:
        return
    for order in (0, 1, 2):  # servers, then batches, then graphs
        for h in list(_live):
            if getattr(h, "_release_order", 2) == order:
                try:
                    h._release()
                except Exception:
                    pass
    _lib.irgl_shutdown()
    _shut = True


atexit.register(_release_all)


def irgl_shutdown() -> int:
    """Return the library's process-lifetime host resources (see irgl.h)."""
    return int(_lib.irgl_shutdown())
_lib.irgl_status_string.restype = ctypes.c_char_p
_lib.irgl_status_string.argtypes = [ctypes.c_int32]
_lib.irgl_last_hip_error.restype = ctypes.c_int32
_lib.irgl_last_hip_error.argtypes = []
_lib.irgl_graph_upload.restype = ctypes.c_int32
_lib.irgl_graph_upload.argtypes = [ctypes.POINTER(irgl_csr), ctypes.POINTER(_c)]
_lib.irgl_reorder_bytes.restype = ctypes.c_int32
_lib.irgl_reorder_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_graph_upload_reordered.restype = ctypes.c_int32
_lib.irgl_graph_upload_reordered.argtypes = [ctypes.POINTER(irgl_csr), _c, ctypes.c_size_t, ctypes.POINTER(_c)]
_lib.irgl_graph_free.restype = ctypes.c_int32
_lib.irgl_graph_free.argtypes = [_c]
_lib.irgl_graph_default_delta.restype = ctypes.c_int32
_lib.irgl_graph_default_delta.argtypes = [_c, ctypes.POINTER(ctypes.c_uint32)]
_lib.irgl_graph_set_delta.restype = ctypes.c_int32
_lib.irgl_graph_set_delta.argtypes = [_c, ctypes.c_uint32]
_lib.irgl_workspace_bytes.restype = ctypes.c_int32
_lib.irgl_workspace_bytes.argtypes = [_c, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(irgl_config),
                                      ctypes.POINTER(ctypes.c_size_t)]
for _name in ("irgl_bfs", "irgl_sssp"):
    _f = getattr(_lib, _name)
    _f.restype = ctypes.c_int32
    _f.argtypes = [_c, ctypes.c_int32, _c, _c, _c, ctypes.c_size_t, _c, _c, ctypes.POINTER(irgl_config)]
_lib.irgl_sssp_noalloc.restype = ctypes.c_int32
_lib.irgl_sssp_noalloc.argtypes = [_c, ctypes.c_int32, _c, _c, _c, _c, ctypes.POINTER(irgl_config)]
_lib.irgl_wallclock_khz.restype = ctypes.c_int32
_lib.irgl_wallclock_khz.argtypes = [ctypes.POINTER(ctypes.c_int32)]
_lib.irgl_query_status.restype = ctypes.c_int32
_lib.irgl_query_status.argtypes = [_c, _c, ctypes.POINTER(irgl_stats)]


class IrglError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = irgl_status_string(status)
        if status == IRGL_ERR_DEVICE:
            msg += f" (hipError {irgl_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]" if where else f"{msg} [{status}]")


def _check(status: int, where: str) -> None:
    if status != IRGL_OK:
        raise IrglError(status, where)


def irgl_version() -> int:
    return int(_lib.irgl_version())


def irgl_status_string(status: int) -> str:
    return _lib.irgl_status_string(int(status)).decode()


def irgl_last_hip_error() -> int:
    return int(_lib.irgl_last_hip_error())


def irgl_wallclock_khz() -> int:
    out = ctypes.c_int32()
    _check(_lib.irgl_wallclock_khz(ctypes.byref(out)), "irgl_wallclock_khz")
    return int(out.value)


def _dev_ptr(t: Optional[torch.Tensor], name: str, dtypes, numel: Optional[int] = None) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device (cuda) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


_I32 = (torch.int32, getattr(torch, "uint32", torch.int32))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_config(cfg=None) -> Optional[irgl_config]:
    """dict / irgl_config / None -> irgl_config (zero fields take defaults)."""
    if cfg is None or isinstance(cfg, irgl_config):
        return cfg
    c = irgl_config()
    for k, v in dict(cfg).items():
        if k in ("abort_flag", "trace"):
            setattr(c, k, v if isinstance(v, int) or v is None else v.data_ptr())
        else:
            setattr(c, k, int(v))
    return c


def _cfg_ptr(cfg):
    c = make_config(cfg)
    return (ctypes.byref(c) if c is not None else None), c


class Graph:
    """A device-resident CSR graph registered with the library.

    Holds references to the borrowed tensors for the handle's lifetime."""

    def __init__(self, handle: int, n: int, m: int, row_ptr, col, w, flags: int, store=None):
        self.handle = handle
        self.n = n
        self.m = m
        self.row_ptr = row_ptr
        self.col = col
        self.w = w
        self.flags = flags
        self.store = store  # device store of a relabelled copy (irgl_graph_upload_reordered)
        _live.add(self)

    _release_order = 2

    @property
    def reordered(self) -> bool:
        return self.store is not None

    @property
    def weighted(self) -> bool:
        return self.w is not None

    def free(self) -> None:
        if self.handle and not _shut:
            _lib.irgl_graph_free(self.handle)
        self.handle = None

    _release = free

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def irgl_graph_upload(row_ptr: torch.Tensor, col: torch.Tensor, w: Optional[torch.Tensor] = None,
                      flags: int = 0) -> Graph:
    """Register a device CSR (int32 row_ptr[n+1], int32 col[m], uint32/int32 w[m] or None)."""
    n = int(row_ptr.numel()) - 1
    m = int(col.numel())
    csr = irgl_csr()
    csr.n = n
    csr.m = m
    csr.row_ptr = _dev_ptr(row_ptr, "row_ptr", _I32)
    csr.col = _dev_ptr(col, "col", _I32) if m > 0 else None
    csr.w = _dev_ptr(w, "w", _I32, m) if w is not None else None
    csr.flags = int(flags)
    h = ctypes.c_void_p()
    _check(_lib.irgl_graph_upload(ctypes.byref(csr), ctypes.byref(h)), "irgl_graph_upload")
    return Graph(h.value, n, m, row_ptr, col, w, flags)


def irgl_reorder_bytes(n: int, m: int, weighted: bool) -> int:
    out = ctypes.c_size_t()
    _check(_lib.irgl_reorder_bytes(int(n), int(m), int(bool(weighted)), ctypes.byref(out)), "irgl_reorder_bytes")
    return int(out.value)


def irgl_graph_upload_reordered(row_ptr: torch.Tensor, col: torch.Tensor, w: Optional[torch.Tensor] = None,
                                flags: int = 0, store: Optional[torch.Tensor] = None) -> Graph:
    """Register a device CSR traversed in a degree-sorted relabelled copy built
    in `store` (allocated here when not given); ids stay the caller's."""
    n = int(row_ptr.numel()) - 1
    m = int(col.numel())
    if store is None:
        store = torch.empty(irgl_reorder_bytes(n, m, w is not None), dtype=torch.uint8, device=row_ptr.device)
    csr = irgl_csr()
    csr.n = n
    csr.m = m
    csr.row_ptr = _dev_ptr(row_ptr, "row_ptr", _I32)
    csr.col = _dev_ptr(col, "col", _I32) if m > 0 else None
    csr.w = _dev_ptr(w, "w", _I32, m) if w is not None else None
    csr.flags = int(flags)
    h = ctypes.c_void_p()
    _check(_lib.irgl_graph_upload_reordered(ctypes.byref(csr), _dev_ptr(store, "store", (torch.uint8,)),
                                            store.numel(), ctypes.byref(h)), "irgl_graph_upload_reordered")
    return Graph(h.value, n, m, row_ptr, col, w, flags, store=store)


def irgl_graph_free(g: Graph) -> None:
    g.free()


def irgl_workspace_bytes(g: Graph, kind: int, with_parent: bool = False, cfg=None) -> int:
    out = ctypes.c_size_t()
    cp, _keep = _cfg_ptr(cfg)
    _check(_lib.irgl_workspace_bytes(g.handle, int(kind), int(bool(with_parent)), cp, ctypes.byref(out)),
           "irgl_workspace_bytes")
    return int(out.value)


def workspace(g: Graph, kind: int, with_parent: bool = False, cfg=None) -> torch.Tensor:
    """Allocate a device workspace tensor of the size the library asks for."""
    nbytes = irgl_workspace_bytes(g, kind, with_parent, cfg)
    return torch.empty(nbytes, dtype=torch.uint8, device=g.row_ptr.device)


def _run(fn, name, g: Graph, src: int, out: torch.Tensor, parent, ws, stream, stats, cfg) -> None:
    if g.handle is None:
        raise ValueError("graph handle was freed")
    op = _dev_ptr(out, "out", _I32, g.n)
    pp = _dev_ptr(parent, "parent", _I32, g.n)
    if ws is None:
        raise ValueError("a workspace tensor is required (see workspace())")
    wp = _dev_ptr(ws, "ws", (torch.uint8,))
    sp = _dev_ptr(stats, "stats", (torch.uint8,), STATS_BYTES) if stats is not None else None
    cp, _keep = _cfg_ptr(cfg)
    _check(fn(g.handle, int(src), op, pp, wp, ws.numel(), _stream_handle(stream), sp, cp), name)


def irgl_bfs(g: Graph, src: int, level: torch.Tensor, parent: Optional[torch.Tensor] = None,
             ws: Optional[torch.Tensor] = None, stream=None, stats: Optional[torch.Tensor] = None,
             cfg=None) -> None:
    """Asynchronous BFS from src on `stream`; level is a device int32/uint32 [n]."""
    _run(_lib.irgl_bfs, "irgl_bfs", g, src, level, parent, ws, stream, stats, cfg)


def irgl_sssp(g: Graph, src: int, dist: torch.Tensor, parent: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None, stream=None, stats: Optional[torch.Tensor] = None,
              cfg=None) -> None:
    """Asynchronous SSSP from src on `stream`; dist is a device int32/uint32 [n]."""
    _run(_lib.irgl_sssp, "irgl_sssp", g, src, dist, parent, ws, stream, stats, cfg)


IRGL_NOALLOC_SCRATCH_BYTES = 64 << 20


def irgl_sssp_noalloc(g: Graph, src: int, dist: torch.Tensor, parent: Optional[torch.Tensor] = None,
                      stream=None, stats: Optional[torch.Tensor] = None, cfg=None) -> None:
    """irgl_sssp on the library's own device scratch (no workspace argument,
    nothing allocated); calls that overlap on one device race."""
    if g.handle is None:
        raise ValueError("graph handle was freed")
    op = _dev_ptr(dist, "dist", _I32, g.n)
    pp = _dev_ptr(parent, "parent", _I32, g.n)
    sp = _dev_ptr(stats, "stats", (torch.uint8,), STATS_BYTES) if stats is not None else None
    cp, _keep = _cfg_ptr(cfg)
    _check(_lib.irgl_sssp_noalloc(g.handle, int(src), op, pp, _stream_handle(stream), sp, cp),
           "irgl_sssp_noalloc")


def irgl_query_status(ws: torch.Tensor, stream=None) -> dict:
    """Synchronize `stream` and return the statistics of the workspace's last query."""
    st = irgl_stats()
    _check(_lib.irgl_query_status(_dev_ptr(ws, "ws", (torch.uint8,)), _stream_handle(stream),
                                  ctypes.byref(st)), "irgl_query_status")
    return st.as_dict()


# ---------------------------------------------------------------------------
# Minimum spanning forest (Boruvka, the Atomic construct's workload).
# ---------------------------------------------------------------------------

IRGL_LOCK_PACKED = 0
IRGL_LOCK_SPIN = 1
IRGL_LOCK_TICKET = 2


class irgl_mst_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("lock", ctypes.c_uint32),
                ("watchdog_ms", ctypes.c_uint32), ("barrier", ctypes.c_uint32)]


_lib.irgl_mst_workspace_bytes.restype = ctypes.c_int32
_lib.irgl_mst_workspace_bytes.argtypes = [_c, ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_mst.restype = ctypes.c_int32
_lib.irgl_mst.argtypes = [_c, _c, _c, _c, _c, ctypes.c_size_t, _c, _c, ctypes.POINTER(irgl_mst_config)]


def _mst_config(cfg):
    if cfg is None or isinstance(cfg, irgl_mst_config):
        return cfg
    c = irgl_mst_config()
    for k, v in dict(cfg).items():
        setattr(c, k, int(v))
    return c


def irgl_mst_workspace_bytes(g: Graph) -> int:
    out = ctypes.c_size_t()
    _check(_lib.irgl_mst_workspace_bytes(g.handle, ctypes.byref(out)), "irgl_mst_workspace_bytes")
    return int(out.value)


def irgl_mst(g: Graph, weight: torch.Tensor, component: Optional[torch.Tensor] = None,
             in_forest: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None,
             stats: Optional[torch.Tensor] = None, cfg=None) -> None:
    """Asynchronous minimum spanning forest on `stream`: weight is a device
    int64/uint64 [1]; component a device int32 [n] or None; in_forest a device
    uint8 [m] or None."""
    if g.handle is None:
        raise ValueError("graph handle was freed")
    wp = _dev_ptr(weight, "weight", (torch.int64, getattr(torch, "uint64", torch.int64)), 1)
    cp_ = _dev_ptr(component, "component", _I32, g.n)
    fp = _dev_ptr(in_forest, "in_forest", (torch.uint8,), int(g.col.numel()))
    if ws is None:
        raise ValueError("a workspace tensor is required (see irgl_mst_workspace_bytes())")
    sp = _dev_ptr(stats, "stats", (torch.uint8,), STATS_BYTES) if stats is not None else None
    c = _mst_config(cfg)
    _check(_lib.irgl_mst(g.handle, wp, cp_, fp, _dev_ptr(ws, "ws", (torch.uint8,)), ws.numel(),
                         _stream_handle(stream), sp, ctypes.byref(c) if c is not None else None), "irgl_mst")


def mst(g: Graph, cfg=None, stream=None):
    """Run irgl_mst synchronously with fresh outputs: (weight, component, in_forest, stats)."""
    dev = g.row_ptr.device
    weight = torch.zeros(1, dtype=torch.int64, device=dev)
    comp = torch.empty(g.n, dtype=torch.int32, device=dev)
    in_forest = torch.empty(int(g.col.numel()), dtype=torch.uint8, device=dev)
    ws = torch.empty(irgl_mst_workspace_bytes(g), dtype=torch.uint8, device=dev)
    stats = stats_tensor(dev)
    irgl_mst(g, weight, comp, in_forest, ws, stream, stats, cfg)
    if stream is not None:
        stream.synchronize()
    st = read_stats(stats)
    if st["status"] != IRGL_OK:
        raise IrglError(st["status"], "device")
    return int(weight.item()), comp, in_forest, st


def stats_tensor(device) -> torch.Tensor:
    """A zeroed device buffer for one irgl_stats."""
    return torch.zeros(STATS_BYTES, dtype=torch.uint8, device=device)


def read_stats(buf: torch.Tensor) -> dict:
    """Decode a device irgl_stats buffer (synchronizes through .cpu())."""
    raw = bytes(buf.cpu().numpy().tobytes())
    st = irgl_stats.from_buffer_copy(raw)
    return st.as_dict()


def read_stats_array(buf: torch.Tensor) -> list:
    """Decode a device [k, STATS_BYTES] array of irgl_stats (one copy)."""
    raw = buf.cpu().numpy()
    return [irgl_stats.from_buffer_copy(bytes(raw[i].tobytes())).as_dict() for i in range(raw.shape[0])]


def as_u32_numpy(t: torch.Tensor):
    """Device int32 tensor holding uint32 bits -> host numpy uint32."""
    return t.cpu().numpy().view("uint32")


# ---------------------------------------------------------------------------
# Convenience: one synchronous query with freshly allocated outputs.
# ---------------------------------------------------------------------------

def query(g: Graph, kind: int, src: int, with_parent: bool = False, cfg=None, stream=None,
          check: bool = True):
    """Run one BFS/SSSP query and wait for it.  Returns (values, parent, stats)."""
    dev = g.row_ptr.device
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    parent = torch.empty(g.n, dtype=torch.int32, device=dev) if with_parent else None
    ws = workspace(g, kind, with_parent, cfg)
    stats = stats_tensor(dev)
    fn = irgl_bfs if kind == IRGL_KIND_BFS else irgl_sssp
    fn(g, src, out, parent, ws, stream, stats, cfg)
    if stream is not None:
        stream.synchronize()
    st = read_stats(stats)
    if check and st["status"] != IRGL_OK:
        raise IrglError(st["status"], "device")
    return out, parent, st


def irgl_graph_default_delta(g: Graph) -> int:
    """The SSSP near/far step a query on g takes when its delta is left at 0."""
    out = ctypes.c_uint32()
    _check(_lib.irgl_graph_default_delta(g.handle, ctypes.byref(out)), "irgl_graph_default_delta")
    return int(out.value)


def irgl_graph_set_delta(g: Graph, delta: int) -> None:
    """Set the default SSSP step of single queries on g (rebuilds the
    light/heavy partition of a relabelled weighted graph; synchronous)."""
    _check(_lib.irgl_graph_set_delta(g.handle, int(delta)), "irgl_graph_set_delta")


def upload(g, flags: int = IRGL_VALIDATE, reorder: bool = False) -> Graph:
    """Register a graphgen.CSRGraph whose tensors are already on the device
    (reorder: traverse a degree-sorted relabelled copy)."""
    fl = flags | (IRGL_SYMMETRIC if getattr(g, "symmetric", False) else 0)
    if reorder:
        return irgl_graph_upload_reordered(g.row_ptr, g.col, g.w, fl)
    return irgl_graph_upload(g.row_ptr, g.col, g.w, fl)


# ---------------------------------------------------------------------------
# Batched queries (irgl_batch_*): many queries in one persistent launch.
# ---------------------------------------------------------------------------

class irgl_task(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("kind", ctypes.c_int32), ("src", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("parent", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class irgl_batch_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("team", ctypes.c_int32), ("t_wave", ctypes.c_int32),
                ("t_block", ctypes.c_int32), ("t_grid", ctypes.c_int32), ("delta", ctypes.c_uint32),
                ("watchdog_ms", ctypes.c_uint32), ("grid", ctypes.c_int32), ("barrier", ctypes.c_uint32),
                ("gang_edges", ctypes.c_uint32), ("gang_queue", ctypes.c_uint32)]


_lib.irgl_control_block_sizes.restype = ctypes.c_int32
_lib.irgl_control_block_sizes.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
_lib.irgl_batch_workspace_bytes.restype = ctypes.c_int32
_lib.irgl_batch_workspace_bytes.argtypes = [ctypes.POINTER(irgl_task), ctypes.c_int32,
                                            ctypes.POINTER(irgl_batch_config), ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_batch_submit.restype = ctypes.c_int32
_lib.irgl_batch_submit.argtypes = [ctypes.POINTER(irgl_task), ctypes.c_int32, _c, ctypes.c_size_t,
                                   ctypes.POINTER(irgl_batch_config), _c, ctypes.POINTER(_c)]
_lib.irgl_batch_wait.restype = ctypes.c_int32
_lib.irgl_batch_wait.argtypes = [_c, ctypes.POINTER(irgl_stats)]
_lib.irgl_batch_free.restype = ctypes.c_int32
_lib.irgl_batch_free.argtypes = [_c]


def irgl_control_block_sizes() -> list:
    """T_control: workgroup sizes both loop bodies support (usable by the batch kernel)."""
    buf = (ctypes.c_int32 * 8)()
    cnt = ctypes.c_int32()
    _check(_lib.irgl_control_block_sizes(buf, 8, ctypes.byref(cnt)), "irgl_control_block_sizes")
    return [int(buf[i]) for i in range(min(cnt.value, 8))]


def make_batch_config(cfg=None) -> Optional[irgl_batch_config]:
    if cfg is None or isinstance(cfg, irgl_batch_config):
        return cfg
    c = irgl_batch_config()
    for k, v in dict(cfg).items():
        setattr(c, k, int(v))
    return c


class Task:
    """One query of a batch: graph, kind, source, device outputs (allocated here
    when not given)."""

    def __init__(self, g: Graph, kind: int, src: int, out: Optional[torch.Tensor] = None,
                 parent: Optional[torch.Tensor] = None, tag: int = 0, with_parent: bool = False):
        dev = g.row_ptr.device
        self.g = g
        self.kind = int(kind)
        self.src = int(src)
        self.out = out if out is not None else torch.empty(g.n, dtype=torch.int32, device=dev)
        if parent is None and with_parent:
            parent = torch.empty(g.n, dtype=torch.int32, device=dev)
        self.parent = parent
        self.tag = int(tag)
        self.stats = None


def _task_array(tasks):
    arr = (irgl_task * len(tasks))()
    for i, t in enumerate(tasks):
        arr[i].g = t.g.handle
        arr[i].kind = t.kind
        arr[i].src = t.src
        arr[i].out = _dev_ptr(t.out, "out", _I32, t.g.n)
        arr[i].parent = _dev_ptr(t.parent, "parent", _I32, t.g.n) if t.parent is not None else None
        arr[i].tag = t.tag
    return arr


def irgl_batch_workspace_bytes(tasks, cfg=None) -> int:
    arr = _task_array(tasks)
    c = make_batch_config(cfg)
    out = ctypes.c_size_t()
    _check(_lib.irgl_batch_workspace_bytes(arr, len(tasks), ctypes.byref(c) if c is not None else None,
                                           ctypes.byref(out)), "irgl_batch_workspace_bytes")
    return int(out.value)


class Batch:
    _release_order = 1

    def __init__(self, handle, tasks, ws):
        self.handle = handle
        self.tasks = tasks
        self.ws = ws
        _live.add(self)

    def free(self):
        if self.handle and not _shut:
            _lib.irgl_batch_free(self.handle)
        self.handle = None

    _release = free

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def irgl_batch_submit(tasks, ws: Optional[torch.Tensor] = None, cfg=None, stream=None) -> Batch:
    """Launch all tasks in one persistent launch (asynchronous on `stream`)."""
    if ws is None:
        ws = torch.empty(irgl_batch_workspace_bytes(tasks, cfg), dtype=torch.uint8,
                         device=tasks[0].g.row_ptr.device)
    arr = _task_array(tasks)
    c = make_batch_config(cfg)
    h = ctypes.c_void_p()
    _check(_lib.irgl_batch_submit(arr, len(tasks), _dev_ptr(ws, "ws", (torch.uint8,)), ws.numel(),
                                  ctypes.byref(c) if c is not None else None, _stream_handle(stream),
                                  ctypes.byref(h)), "irgl_batch_submit")
    return Batch(h.value, list(tasks), ws)


def irgl_batch_wait(b: Batch) -> list:
    """Wait for the batch; returns per-task statistics (task order) and sets task.stats."""
    st = (irgl_stats * len(b.tasks))()
    _check(_lib.irgl_batch_wait(b.handle, st), "irgl_batch_wait")
    out = [st[i].as_dict() for i in range(len(b.tasks))]
    for t, s in zip(b.tasks, out):
        t.stats = s
    return out


def irgl_batch_free(b: Batch) -> None:
    b.free()


# ---------------------------------------------------------------------------
# Open batches / serving (irgl_batch_open / _enqueue / _poll / _close).
# ---------------------------------------------------------------------------

_lib.irgl_batch_open_bytes.restype = ctypes.c_int32
_lib.irgl_batch_open_bytes.argtypes = [ctypes.POINTER(_c), ctypes.c_int32, ctypes.POINTER(irgl_batch_config),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_batch_open.restype = ctypes.c_int32
_lib.irgl_batch_open.argtypes = [ctypes.POINTER(_c), ctypes.c_int32, ctypes.POINTER(irgl_batch_config),
                                 ctypes.c_int32, ctypes.c_uint32, _c, ctypes.c_size_t, _c, ctypes.POINTER(_c)]
_lib.irgl_batch_enqueue.restype = ctypes.c_int32
_lib.irgl_batch_enqueue.argtypes = [_c, ctypes.POINTER(irgl_task), ctypes.POINTER(ctypes.c_uint64)]
_lib.irgl_batch_poll.restype = ctypes.c_int32
_lib.irgl_batch_poll.argtypes = [_c, ctypes.c_uint64, ctypes.POINTER(irgl_stats), ctypes.POINTER(ctypes.c_int32)]
_lib.irgl_batch_close.restype = ctypes.c_int32
_lib.irgl_batch_close.argtypes = [_c]
_lib.irgl_batch_launches.restype = ctypes.c_int32
_lib.irgl_batch_launches.argtypes = [_c, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]


def _graph_array(graphs):
    arr = (ctypes.c_void_p * len(graphs))()
    for i, g in enumerate(graphs):
        arr[i] = g.handle
    return arr


def irgl_batch_open_bytes(graphs, cfg=None, ring_cap: int = 256) -> int:
    c = make_batch_config(cfg)
    out = ctypes.c_size_t()
    _check(_lib.irgl_batch_open_bytes(_graph_array(graphs), len(graphs),
                                      ctypes.byref(c) if c is not None else None, int(ring_cap),
                                      ctypes.byref(out)), "irgl_batch_open_bytes")
    return int(out.value)


class Server:
    """An open batch: tasks are enqueued while the server kernel runs."""

    _release_order = 0

    def __init__(self, handle, graphs, ws, stream):
        self.handle = handle
        self.graphs = list(graphs)
        self.ws = ws
        self.stream = stream
        self.inflight = {}
        _live.add(self)

    def close(self):
        if self.handle and not _shut:
            _lib.irgl_batch_close(self.handle)
        self.handle = None

    _release = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def irgl_batch_open(graphs, cfg=None, ring_cap: int = 256, idle_ms: int = 50, ws=None, stream=None) -> Server:
    """The server kernel keeps its stream busy while it runs, so by default it
    gets a stream of its own (default priority), ordered after the caller's
    current stream.  Task buffers are written as soon as a task is queued: the
    caller finishes its own pending work on them first."""
    dev = graphs[0].row_ptr.device
    if ws is None:
        ws = torch.empty(irgl_batch_open_bytes(graphs, cfg, ring_cap), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.Stream(device=dev)
        stream.wait_stream(torch.cuda.current_stream(dev))
    c = make_batch_config(cfg)
    h = ctypes.c_void_p()
    _check(_lib.irgl_batch_open(_graph_array(graphs), len(graphs), ctypes.byref(c) if c is not None else None,
                                int(ring_cap), int(idle_ms), _dev_ptr(ws, "ws", (torch.uint8,)), ws.numel(),
                                _stream_handle(stream), ctypes.byref(h)), "irgl_batch_open")
    return Server(h.value, graphs, ws, stream)


def irgl_batch_enqueue(s: Server, task: Task):
    """Queue a task; returns its ticket, or None when the ring is full (BUSY)."""
    arr = _task_array([task])
    t = ctypes.c_uint64()
    st = _lib.irgl_batch_enqueue(s.handle, arr, ctypes.byref(t))
    if st == IRGL_ERR_BUSY:
        return None
    _check(st, "irgl_batch_enqueue")
    s.inflight[int(t.value)] = task
    return int(t.value)


def irgl_batch_poll(s: Server, ticket: int):
    """Statistics dict when the task has finished, else None."""
    st = irgl_stats()
    done = ctypes.c_int32()
    _check(_lib.irgl_batch_poll(s.handle, int(ticket), ctypes.byref(st), ctypes.byref(done)), "irgl_batch_poll")
    if done.value:
        task = s.inflight.pop(int(ticket), None)
        d = st.as_dict()
        if task is not None:
            task.stats = d
        return d
    return None


def irgl_batch_launches(s: Server):
    """(server kernel launches so far, launches that gave up at their start check)."""
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_lib.irgl_batch_launches(s.handle, ctypes.byref(a), ctypes.byref(b)), "irgl_batch_launches")
    return int(a.value), int(b.value)


def irgl_batch_close(s: Server) -> None:
    s.close()


# ---------------------------------------------------------------------------
# Pipes (irgl_pipe_*): orchestration programs run by one outlined control
# kernel over the shared in / out / retry worklists.
# ---------------------------------------------------------------------------

IRGL_PIPE_INVOKE, IRGL_PIPE_ITERATE, IRGL_PIPE_BEGIN, IRGL_PIPE_END = 0, 1, 2, 3
IRGL_PIPE_IF, IRGL_PIPE_JUMP, IRGL_PIPE_INIT_SOURCE = 4, 5, 6
IRGL_COND_IN_EMPTY, IRGL_COND_FRONTIER_LARGE, IRGL_COND_RETURNED = 0, 1, 2
IRGL_COND_NOT = 0x100
(IRGL_BODY_BFS_PUSH, IRGL_BODY_BFS_PULL, IRGL_BODY_MST_INIT, IRGL_BODY_MST_FINDMIN, IRGL_BODY_MST_HOOK,
 IRGL_BODY_MST_JUMP, IRGL_BODY_MST_RELABEL, IRGL_BODY_MST_MINID, IRGL_BODY_MST_LABEL) = range(9)
IRGL_BODY_COUNT = 9
IRGL_BLOCK_ELASTIC, IRGL_BLOCK_SHRINKABLE, IRGL_BLOCK_FIXED = 0, 1, 2


class irgl_block_constraint(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("block", ctypes.c_int32), ("lds_base", ctypes.c_int32),
                ("lds_per_thread", ctypes.c_int32)]


class irgl_pipe_op(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class irgl_pipe_io(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("level", ctypes.c_void_p), ("component", ctypes.c_void_p),
                ("in_forest", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("trace", ctypes.c_void_p),
                ("trace_len", ctypes.c_uint32), ("block", ctypes.c_int32), ("max_invocations", ctypes.c_uint32),
                ("watchdog_ms", ctypes.c_uint32), ("grid", ctypes.c_int32), ("force_retry", ctypes.c_uint32)]


_lib.irgl_control_block.restype = ctypes.c_int32
_lib.irgl_control_block.argtypes = [ctypes.POINTER(irgl_block_constraint), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32)]
_lib.irgl_pipe_body_constraint.restype = ctypes.c_int32
_lib.irgl_pipe_body_constraint.argtypes = [ctypes.c_int32, ctypes.POINTER(irgl_block_constraint)]
_lib.irgl_pipe_check.restype = ctypes.c_int32
_lib.irgl_pipe_check.argtypes = [ctypes.POINTER(irgl_pipe_op), ctypes.c_int32]
_lib.irgl_pipe_control_block.restype = ctypes.c_int32
_lib.irgl_pipe_control_block.argtypes = [ctypes.POINTER(irgl_pipe_op), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.irgl_pipe_workspace_bytes.restype = ctypes.c_int32
_lib.irgl_pipe_workspace_bytes.argtypes = [_c, ctypes.POINTER(irgl_pipe_op), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_pipe_run.restype = ctypes.c_int32
_lib.irgl_pipe_run.argtypes = [_c, ctypes.POINTER(irgl_pipe_op), ctypes.c_int32, ctypes.POINTER(irgl_pipe_io), _c,
                               ctypes.c_size_t, _c, _c]


def _program(ops):
    arr = (irgl_pipe_op * len(ops))()
    for i, o in enumerate(ops):
        o = tuple(o) + (0,) * (3 - len(o))
        arr[i].op, arr[i].a, arr[i].b = int(o[0]), int(o[1]), int(o[2])
    return arr


def irgl_control_block(constraints, lds_limit: int) -> int:
    """T_control of (kind, block, lds_base, lds_per_thread) tuples; raises on an empty set."""
    arr = (irgl_block_constraint * max(1, len(constraints)))()
    for i, c in enumerate(constraints):
        arr[i].kind, arr[i].block, arr[i].lds_base, arr[i].lds_per_thread = (int(x) for x in c)
    out = ctypes.c_int32()
    _check(_lib.irgl_control_block(arr, len(constraints), int(lds_limit), ctypes.byref(out)), "irgl_control_block")
    return int(out.value)


def irgl_pipe_body_constraint(body: int):
    c = irgl_block_constraint()
    _check(_lib.irgl_pipe_body_constraint(int(body), ctypes.byref(c)), "irgl_pipe_body_constraint")
    return (c.kind, c.block, c.lds_base, c.lds_per_thread)


def irgl_pipe_check(ops) -> None:
    arr = _program(ops)
    _check(_lib.irgl_pipe_check(arr, len(ops)), "irgl_pipe_check")


def irgl_pipe_control_block(ops, requested: int = 0, lds_limit: int = 0) -> int:
    arr = _program(ops)
    out = ctypes.c_int32()
    _check(_lib.irgl_pipe_control_block(arr, len(ops), int(requested), int(lds_limit), ctypes.byref(out)),
           "irgl_pipe_control_block")
    return int(out.value)


def irgl_pipe_workspace_bytes(g: Graph, ops) -> int:
    arr = _program(ops)
    out = ctypes.c_size_t()
    _check(_lib.irgl_pipe_workspace_bytes(g.handle, arr, len(ops), ctypes.byref(out)), "irgl_pipe_workspace_bytes")
    return int(out.value)


def irgl_pipe_run(g: Graph, ops, src: int = 0, level=None, component=None, in_forest=None, weight=None,
                  trace=None, block: int = 0, max_invocations: int = 0, grid: int = 0, ws=None, stream=None,
                  stats=None, force_retry: bool = False):
    """Run a pipe program on g (asynchronous on `stream`)."""
    arr = _program(ops)
    if ws is None:
        ws = torch.empty(irgl_pipe_workspace_bytes(g, ops), dtype=torch.uint8, device=g.row_ptr.device)
    io = irgl_pipe_io()
    io.src = int(src)
    io.level = _dev_ptr(level, "level", _I32, g.n)
    io.component = _dev_ptr(component, "component", _I32, g.n)
    io.in_forest = _dev_ptr(in_forest, "in_forest", (torch.uint8,), g.m) if in_forest is not None else None
    io.weight = _dev_ptr(weight, "weight", (torch.int64,), 1)
    io.trace = _dev_ptr(trace, "trace", _I32)
    io.trace_len = int(trace.numel()) if trace is not None else 0
    io.block = int(block)
    io.max_invocations = int(max_invocations)
    io.grid = int(grid)
    io.force_retry = 1 if force_retry else 0
    sp = _dev_ptr(stats, "stats", (torch.uint8,), STATS_BYTES) if stats is not None else None
    _check(_lib.irgl_pipe_run(g.handle, arr, len(ops), ctypes.byref(io), _dev_ptr(ws, "ws", (torch.uint8,)),
                              ws.numel(), _stream_handle(stream), sp), "irgl_pipe_run")
    return ws


def pipe_bfs_program():
    """BFS whose every level is consumed by the top-down or the bottom-up body,
    chosen at run time by the size of the frontier (dynamic piping)."""
    return [(IRGL_PIPE_INIT_SOURCE,),
            (IRGL_PIPE_BEGIN, 0),
            (IRGL_PIPE_IF, IRGL_COND_FRONTIER_LARGE, 5),
            (IRGL_PIPE_INVOKE, IRGL_BODY_BFS_PULL),
            (IRGL_PIPE_JUMP, 6),
            (IRGL_PIPE_INVOKE, IRGL_BODY_BFS_PUSH),
            (IRGL_PIPE_END,)]


def pipe_boruvka_program():
    """Boruvka minimum spanning forest as a Pipe Once around a looping Pipe:
    find-min-edge (non-blocking Atomic, Else -> retry), hook, Iterate pointer
    jumping, relabel; then the smallest id of every tree."""
    return [(IRGL_PIPE_BEGIN, 1),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_INIT),
            (IRGL_PIPE_BEGIN, 0),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_FINDMIN),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_HOOK),
            (IRGL_PIPE_ITERATE, IRGL_BODY_MST_JUMP),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_RELABEL),
            (IRGL_PIPE_END,),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_MINID),
            (IRGL_PIPE_INVOKE, IRGL_BODY_MST_LABEL),
            (IRGL_PIPE_END,)]


# ---------------------------------------------------------------------------
# Delaunay mesh refinement (the Exclusive construct's workload).
# ---------------------------------------------------------------------------

class irgl_mesh(ctypes.Structure):
    _fields_ = [("pts", ctypes.c_void_p), ("tri", ctypes.c_void_p), ("nbr", ctypes.c_void_p),
                ("npts", ctypes.c_int32), ("ntri", ctypes.c_int32), ("pcap", ctypes.c_int32),
                ("tcap", ctypes.c_int32)]


class irgl_dmr_config(ctypes.Structure):
    _fields_ = [("min_angle", ctypes.c_double), ("block", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("max_invocations", ctypes.c_uint32), ("watchdog_ms", ctypes.c_uint32),
                ("barrier", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class irgl_dmr_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("invocations", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("refined", ctypes.c_uint64), ("conflicts", ctypes.c_uint64), ("inserted", ctypes.c_uint32),
                ("splits", ctypes.c_uint32), ("npts", ctypes.c_int32), ("ntri", ctypes.c_int32),
                ("final_bad", ctypes.c_uint32), ("max_cavity", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


DMR_STATS_BYTES = ctypes.sizeof(irgl_dmr_stats)

_lib.irgl_dmr_workspace_bytes.restype = ctypes.c_int32
_lib.irgl_dmr_workspace_bytes.argtypes = [ctypes.POINTER(irgl_mesh), ctypes.POINTER(ctypes.c_size_t)]
_lib.irgl_dmr_refine.restype = ctypes.c_int32
_lib.irgl_dmr_refine.argtypes = [ctypes.POINTER(irgl_mesh), _c, ctypes.c_size_t, ctypes.POINTER(irgl_dmr_config),
                                 _c, _c]


class DeviceMesh:
    """A mesh resident on the device (tensors owned here): pts float64
    [pcap, 2], tri and nbr int32 [tcap, 4], plus the counts in use."""

    def __init__(self, pts: torch.Tensor, tri: torch.Tensor, nbr: torch.Tensor, npts: int, ntri: int):
        self.pts, self.tri, self.nbr = pts, tri, nbr
        self.npts, self.ntri = int(npts), int(ntri)

    @classmethod
    def from_host(cls, m, device) -> "DeviceMesh":
        """From a meshgen.Mesh (host arrays sized to their capacities)."""
        return cls(torch.from_numpy(m.pts).to(device), torch.from_numpy(m.tri).to(device),
                   torch.from_numpy(m.nbr).to(device), m.npts, m.ntri)

    def c_struct(self) -> irgl_mesh:
        s = irgl_mesh()
        s.pts = _dev_ptr(self.pts, "pts", (torch.float64,))
        s.tri = _dev_ptr(self.tri, "tri", (torch.int32,))
        s.nbr = _dev_ptr(self.nbr, "nbr", (torch.int32,))
        if self.pts.dim() != 2 or self.pts.shape[1] != 2:
            raise ValueError("pts must be [pcap, 2]")
        if self.tri.dim() != 2 or self.tri.shape[1] != 4 or self.nbr.shape != self.tri.shape:
            raise ValueError("tri and nbr must be [tcap, 4]")
        s.npts, s.ntri = self.npts, self.ntri
        s.pcap, s.tcap = int(self.pts.shape[0]), int(self.tri.shape[0])
        return s


def _dmr_config(cfg):
    if cfg is None or isinstance(cfg, irgl_dmr_config):
        return cfg
    c = irgl_dmr_config()
    for k, v in dict(cfg).items():
        setattr(c, k, float(v) if k == "min_angle" else int(v))
    return c


def irgl_dmr_workspace_bytes(mesh: DeviceMesh) -> int:
    out = ctypes.c_size_t()
    s = mesh.c_struct()
    _check(_lib.irgl_dmr_workspace_bytes(ctypes.byref(s), ctypes.byref(out)), "irgl_dmr_workspace_bytes")
    return int(out.value)


def irgl_dmr_refine(mesh: DeviceMesh, ws: torch.Tensor, cfg=None, stream=None,
                    stats: Optional[torch.Tensor] = None) -> None:
    """Asynchronous refinement of `mesh` in place on `stream`."""
    s = mesh.c_struct()
    c = _dmr_config(cfg)
    sp = _dev_ptr(stats, "stats", (torch.uint8,), DMR_STATS_BYTES) if stats is not None else None
    _check(_lib.irgl_dmr_refine(ctypes.byref(s), _dev_ptr(ws, "ws", (torch.uint8,)), ws.numel(),
                                ctypes.byref(c) if c is not None else None, _stream_handle(stream), sp),
           "irgl_dmr_refine")


def read_dmr_stats(buf: torch.Tensor) -> dict:
    raw = bytes(buf.cpu().numpy().tobytes())
    return irgl_dmr_stats.from_buffer_copy(raw).as_dict()


def dmr(mesh: DeviceMesh, cfg=None, stream=None) -> dict:
    """Refine synchronously; updates mesh.npts / mesh.ntri and returns the
    statistics (raises IrglError on a device-side error)."""
    dev = mesh.pts.device
    ws = torch.empty(irgl_dmr_workspace_bytes(mesh), dtype=torch.uint8, device=dev)
    stats = torch.zeros(DMR_STATS_BYTES, dtype=torch.uint8, device=dev)
    irgl_dmr_refine(mesh, ws, cfg, stream, stats)
    if stream is not None:
        stream.synchronize()
    st = read_dmr_stats(stats)
    if st["status"] != IRGL_OK:
        raise IrglError(st["status"], "device")
    mesh.npts, mesh.ntri = st["npts"], st["ntri"]
    return st
