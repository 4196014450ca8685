"""Seeded synthetic graph inputs in CSR form.

This module is the only code shared by the HIP path's callers (tests, bench,
smoke) and the CPU oracle.  It builds graph topology, edge weights and query
sources; it holds none of the traversal arithmetic (no levels, no distances,
no relaxation).

The paper's BFS kernel (Section 4.1, the level-by-level worklist listing)
reads a graph through ``graph.edges(n)`` and ``e.dst``; here that graph is a
compressed-sparse-row structure of three arrays:

* ``row_ptr`` int32[n+1], monotone, ``row_ptr[0] == 0``, ``row_ptr[n] == m``;
* ``col``     int32[m], neighbours of each vertex sorted ascending;
* ``w``       int32[m] holding uint32 weights >= 1 (``None`` when unweighted).

Randomness is counter based: every random 32-bit word is a hash of
``(seed, stream, index)`` computed with 64-bit integer tensor arithmetic that
never overflows, so the same call gives byte-identical graphs on the CPU and
on a GPU device.  The hash is the "lowbias32" integer mixer (two
xor-shift-multiply rounds) published by C. Wellons; it is used here purely as
a source of uniform bits for input generation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import torch

MASK32 = 0xFFFFFFFF

# Stream identifiers keep independent draws apart for one seed.
_S_RMAT = 0x100          # + level
_S_PERM = 0x200
_S_WEIGHT = 0x300
_S_SOURCE = 0x400
_S_DROP = 0x500
_S_LONG_U = 0x600
_S_LONG_V = 0x601
_S_UNI_U = 0x700
_S_UNI_V = 0x701
_S_C4_N = 0x800
_S_C4_D = 0x801


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2^32 for int64 tensors holding values in [0, 2^32)."""
    lo = x & 0xFFFF
    hi = x >> 16
    return (lo * c + (((hi * c) & 0xFFFF) << 16)) & MASK32


def _mix32(x: torch.Tensor) -> torch.Tensor:
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def _key(seed: int, stream: int) -> int:
    t = torch.tensor([(seed * 0x9E3779B9 + stream * 0x85EBCA6B) & MASK32], dtype=torch.int64)
    t = _mix32(t ^ (stream & MASK32))
    return int(_mix32(t ^ (seed & MASK32)).item())


def rand_u32(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform 32-bit words (as int64) for counters ``idx`` (int64, < 2^32)."""
    k = _key(seed, stream)
    return _mix32((idx + k) & MASK32)


def rand_below(seed: int, stream: int, idx: torch.Tensor, bound: int) -> torch.Tensor:
    """Integers in [0, bound) by multiply-shift of a 32-bit word (bound < 2^31)."""
    assert 0 < bound < (1 << 31)
    return (rand_u32(seed, stream, idx) * bound) >> 32


@dataclasses.dataclass
class CSRGraph:
    """A CSR graph plus the metadata of the recipe that made it."""

    n: int
    row_ptr: torch.Tensor           # int32 [n+1]
    col: torch.Tensor               # int32 [m]
    w: Optional[torch.Tensor]       # int32 [m] (uint32 bit pattern) or None
    name: str = ""
    symmetric: bool = False
    sources: Optional[List[int]] = None

    @property
    def m(self) -> int:
        return int(self.col.numel())

    def to(self, device) -> "CSRGraph":
        return dataclasses.replace(
            self,
            row_ptr=self.row_ptr.to(device),
            col=self.col.to(device),
            w=None if self.w is None else self.w.to(device),
        )

    def numpy(self):
        """Host copies as numpy arrays: (row_ptr int32, col int32, w uint32 | None)."""
        rp = self.row_ptr.cpu().numpy()
        c = self.col.cpu().numpy()
        w = None if self.w is None else self.w.cpu().numpy().view("uint32")
        return rp, c, w


def _csr_from_directed(n: int, src: torch.Tensor, dst: torch.Tensor,
                       w: Optional[torch.Tensor]) -> tuple:
    """Sort directed edges by (src, dst) and build row_ptr/col/w."""
    key = src.to(torch.int64) * n + dst.to(torch.int64)
    order = torch.argsort(key)
    src_s = src[order]
    col = dst[order].to(torch.int32)
    ww = None if w is None else w[order].to(torch.int32)
    counts = torch.bincount(src_s.to(torch.int64), minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=src.device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr.to(torch.int32), col, ww


def _undirected_unique(n: int, u: torch.Tensor, v: torch.Tensor):
    """Drop self-loops, orient as (min, max), deduplicate; sorted ascending."""
    keep = u != v
    u = u[keep]
    v = v[keep]
    a = torch.minimum(u, v).to(torch.int64)
    b = torch.maximum(u, v).to(torch.int64)
    key = torch.unique(a * n + b, sorted=True)
    return key // n, key % n


def _symmetric_graph(n: int, a: torch.Tensor, b: torch.Tensor, weight_seed: Optional[int],
                     wmax: int, name: str) -> CSRGraph:
    """Mirror a deduplicated undirected edge list (a < b) into a symmetric CSR.

    One weight is drawn per undirected edge, after deduplication, indexed by
    the edge's rank in the sorted unique list, and used in both directions.
    """
    mu = a.numel()
    w = None
    if weight_seed is not None:
        idx = torch.arange(mu, dtype=torch.int64, device=a.device)
        w1 = rand_below(weight_seed, _S_WEIGHT, idx, wmax) + 1
        w = torch.cat([w1, w1])
    src = torch.cat([a, b])
    dst = torch.cat([b, a])
    rp, col, ww = _csr_from_directed(n, src, dst, w)
    return CSRGraph(n=n, row_ptr=rp, col=col, w=ww, name=name, symmetric=True)


def pick_sources(g: CSRGraph, k: int, seed: int) -> List[int]:
    """k distinct non-isolated vertices, ordered by a seeded hash of their id."""
    deg = (g.row_ptr[1:] - g.row_ptr[:-1]).to(torch.int64)
    cand = torch.nonzero(deg > 0).flatten()
    if cand.numel() == 0:
        return []
    assert g.n < (1 << 30)
    h = rand_u32(seed, _S_SOURCE, cand)
    order = torch.argsort(h * (g.n + 1) + cand)  # by hash, ties by id
    return [int(x) for x in cand[order[:k]].cpu().tolist()]


# ----------------------------------------------------------------------------
# Recipes
# ----------------------------------------------------------------------------

def grid2d(width: int, height: Optional[int] = None, *, weight_seed: Optional[int] = None,
           wmax: int = 100, drop_p: float = 0.0, long_frac: float = 0.0, seed: int = 0,
           device="cpu") -> CSRGraph:
    """4-neighbour undirected grid, vertex id = row * width + col.

    ``drop_p`` removes each grid edge independently; ``long_frac`` adds
    round(long_frac * #grid edges) uniform random vertex pairs (the road-like
    recipe); the union is deduplicated before weights are drawn.
    """
    height = width if height is None else height
    n = width * height
    ids = torch.arange(n, dtype=torch.int64, device=device)
    r = ids // width
    c = ids % width
    right = ids[c < width - 1]
    down = ids[r < height - 1]
    a = torch.cat([right, down])
    b = torch.cat([right + 1, down + width])
    n_grid = a.numel()
    if drop_p > 0.0:
        thr = int(round(drop_p * 2 ** 32))
        keep = rand_u32(seed, _S_DROP, torch.arange(n_grid, dtype=torch.int64, device=device)) >= thr
        a = a[keep]
        b = b[keep]
    if long_frac > 0.0:
        nl = int(round(long_frac * n_grid))
        idx = torch.arange(nl, dtype=torch.int64, device=device)
        lu = rand_below(seed, _S_LONG_U, idx, n)
        lv = rand_below(seed, _S_LONG_V, idx, n)
        a = torch.cat([a, lu])
        b = torch.cat([b, lv])
    a, b = _undirected_unique(n, a, b)
    name = f"grid{width}x{height}"
    if drop_p or long_frac:
        name += f"_drop{drop_p}_long{long_frac}_s{seed}"
    return _symmetric_graph(n, a, b, weight_seed, wmax, name)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         *, seed: int, weight_seed: Optional[int] = None, wmax: int = 255, relabel: bool = True,
         device="cpu") -> CSRGraph:
    """R-MAT generator: edge_factor * 2^scale tuples, each choosing one of four
    quadrants per bit level with probabilities (a, b, c, 1-a-b-c); then an
    optional seeded vertex relabelling, self-loop removal, symmetrization and
    deduplication, and one uniform weight in [1, wmax] per undirected edge."""
    n = 1 << scale
    assert scale <= 29
    mt = edge_factor * n
    assert mt < (1 << 32)
    ta = int(a * 2 ** 32)
    tab = int((a + b) * 2 ** 32)
    tabc = int((a + b + c) * 2 ** 32)
    idx = torch.arange(mt, dtype=torch.int64, device=device)
    u = torch.zeros(mt, dtype=torch.int64, device=device)
    v = torch.zeros(mt, dtype=torch.int64, device=device)
    for lvl in range(scale):
        x = rand_u32(seed, _S_RMAT + lvl, idx)
        bit_u = (x >= tab).to(torch.int64)                       # quadrants c, d
        bit_v = ((x >= ta) & (x < tab)).to(torch.int64) | (x >= tabc).to(torch.int64)  # b, d
        u = (u << 1) | bit_u
        v = (v << 1) | bit_v
        del x, bit_u, bit_v
    del idx
    if relabel:
        ids = torch.arange(n, dtype=torch.int64, device=device)
        h = rand_u32(seed, _S_PERM, ids)
        order = torch.argsort(h * n + ids)
        label = torch.empty(n, dtype=torch.int64, device=device)
        label[order] = ids
        u = label[u]
        v = label[v]
    ua, va = _undirected_unique(n, u, v)
    del u, v
    g = _symmetric_graph(n, ua, va, weight_seed, wmax, f"rmat{scale}_ef{edge_factor}_s{seed}")
    return g


def uniform_random(n: int, mean_degree: float, *, seed: int, weight_seed: Optional[int] = None,
                   wmax: int = 1000, device="cpu") -> CSRGraph:
    """round(n * mean_degree / 2) uniform random vertex pairs, self-loops removed,
    deduplicated, symmetrized."""
    k = int(round(n * mean_degree / 2))
    idx = torch.arange(k, dtype=torch.int64, device=device)
    u = rand_below(seed, _S_UNI_U, idx, n)
    v = rand_below(seed, _S_UNI_V, idx, n)
    a, b = _undirected_unique(n, u, v)
    return _symmetric_graph(n, a, b, weight_seed, wmax, f"uniform{n}_d{mean_degree}_s{seed}")


def random_directed(n: int, m: int, *, seed: int, weight_seed: Optional[int] = None,
                    wmax: int = 100, allow_self: bool = True, device="cpu") -> CSRGraph:
    """m uniform random directed edges (self-loops and multi-edges kept unless
    ``allow_self`` is False); for tests of the general directed case."""
    idx = torch.arange(m, dtype=torch.int64, device=device)
    u = rand_below(seed, _S_UNI_U, idx, n)
    v = rand_below(seed, _S_UNI_V, idx, n)
    if not allow_self:
        keep = u != v
        u, v, idx = u[keep], v[keep], idx[keep]
    w = None
    if weight_seed is not None:
        w = rand_below(weight_seed, _S_WEIGHT, idx, wmax) + 1
    rp, col, ww = _csr_from_directed(n, u, v, w)
    return CSRGraph(n=n, row_ptr=rp, col=col, w=ww, name=f"directed{n}_{m}_s{seed}")


def from_edges(n: int, src: Sequence[int], dst: Sequence[int], w: Optional[Sequence[int]] = None,
               name: str = "edges") -> CSRGraph:
    """CSR from an explicit directed edge list (kept as given, sorted by (src, dst))."""
    s = torch.as_tensor(list(src), dtype=torch.int64)
    d = torch.as_tensor(list(dst), dtype=torch.int64)
    ww = None if w is None else torch.as_tensor(list(w), dtype=torch.int64)
    rp, col, wt = _csr_from_directed(n, s, d, ww)
    return CSRGraph(n=n, row_ptr=rp, col=col, w=wt, name=name)


# ----------------------------------------------------------------------------
# The five workload configurations
# ----------------------------------------------------------------------------

def config_grid64(device="cpu") -> CSRGraph:
    """64x64 4-neighbour undirected grid, weights U[1,100] (seed 101), source 0."""
    g = grid2d(64, weight_seed=101, wmax=100, device=device)
    g.sources = [0]
    g.name = "grid64x64"
    return g


def config_rmat22(device="cpu", scale: int = 22, nsources: int = 64) -> CSRGraph:
    """RMAT scale 22, edge factor 16, (.57,.19,.19,.05), symmetrized, deduplicated,
    no self-loops, weights U[1,255]; 64 seeded non-isolated sources."""
    g = rmat(scale, 16, 0.57, 0.19, 0.19, seed=scale, weight_seed=scale * 100 + 1, wmax=255,
             device=device)
    g.sources = pick_sources(g, nsources, seed=scale * 100 + 2)
    return g


def config_road(device="cpu", width: int = 4096, long_edges: bool = True) -> CSRGraph:
    """Road-like width x width grid: 5% of grid edges dropped, plus 1% random long
    edges (of the grid-edge count), weights U[1,10000]; source 0 plus 8 random."""
    g = grid2d(width, weight_seed=width + 1, wmax=10000, drop_p=0.05,
               long_frac=0.01 if long_edges else 0.0, seed=width, device=device)
    g.sources = [0] + [s for s in pick_sources(g, 9, seed=width + 2) if s != 0][:8]
    g.name = f"road{width}" + ("" if long_edges else "_nolong")
    return g


def config_batch_sizes(count: int = 256, seed: int = 256):
    """(n_i, mean degree d_i) for the batched workload: n log-uniform in
    [2^12, 2^20], d uniform in [4, 32]."""
    idx = torch.arange(count, dtype=torch.int64)
    un = rand_u32(seed, _S_C4_N, idx).to(torch.float64) / 2 ** 32
    ud = rand_u32(seed, _S_C4_D, idx).to(torch.float64) / 2 ** 32
    ns = [int(round(2 ** (12 + 8 * float(x)))) for x in un]
    ds = [4.0 + 28.0 * float(x) for x in ud]
    return list(zip(ns, ds))


def config_batch(count: int = 256, seed: int = 256, device="cpu", scale_cap: Optional[int] = None):
    """The batched workload's uniform graphs: kind BFS for even i, SSSP for odd i,
    one random non-isolated source each.  Returns a list of (graph, kind, src)."""
    out = []
    for i, (n, d) in enumerate(config_batch_sizes(count, seed)):
        if scale_cap is not None:
            n = min(n, 1 << scale_cap)
        g = uniform_random(n, d, seed=seed * 1000 + i, weight_seed=seed * 1000 + 500 + i,
                           wmax=1000, device=device)
        srcs = pick_sources(g, 1, seed=seed * 1000 + 900 + i)
        out.append((g, "bfs" if i % 2 == 0 else "sssp", srcs[0] if srcs else 0))
    return out


def graph_bytes(g: CSRGraph) -> int:
    return 4 * (g.n + 1) + 4 * g.m + (0 if g.w is None else 4 * g.m)


def log2_ceil(x: int) -> int:
    return 0 if x <= 1 else int(math.ceil(math.log2(x)))
