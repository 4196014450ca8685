"""Named synthetic workloads and a binary CSR file format for the native runner.

Workloads (all seeded, see graphgen):
  grid64          64x64 4-neighbour grid, weights U[1,100], source 0
  rmat22 / rmat20 R-MAT scale 22 / 20, edge factor 16, (.57,.19,.19,.05),
                  symmetrized, weights U[1,255], 64 seeded non-isolated sources
  road4096        4096^2 road-like grid (5% edges dropped, 1% long edges),
                  weights U[1,10000], source 0 + 8 random
  road4096_nolong the same without long edges (high diameter)

File format (little endian): b"IRGLCSR1", int64 n, int64 m, int64 flags
(bit 0: weights present, bit 1: symmetric), int64 nsrc, int32 row_ptr[n+1],
int32 col[m], uint32 w[m] (if bit 0), int32 sources[nsrc].
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

MAGIC = b"IRGLCSR1"


def make_workload(name: str, device, nsources: int = 64):
    from . import graphgen as gg
    if name == "rmat22":
        g = gg.config_rmat22(device=device, nsources=nsources)
    elif name == "rmat20":
        g = gg.config_rmat22(device=device, scale=20, nsources=nsources)
    elif name.startswith("rmat") and name[4:].isdigit():
        g = gg.config_rmat22(device=device, scale=int(name[4:]), nsources=nsources)
    elif name == "grid64":
        g = gg.config_grid64(device=device)
    elif name == "road4096":
        g = gg.config_road(device=device)
    elif name == "road4096_nolong":
        g = gg.config_road(device=device, long_edges=False)
    elif name.startswith("road") and name[4:].isdigit():
        g = gg.config_road(device=device, width=int(name[4:]))
    else:
        raise ValueError(f"unknown workload {name}")
    if g.sources and nsources and len(g.sources) > nsources:
        g.sources = g.sources[:nsources]
    return g


def write_csr(path: str, g) -> None:
    rp, col, w = g.numpy()
    src = np.asarray(g.sources or [0], dtype=np.int32)
    with open(path, "wb") as f:
        f.write(MAGIC)
        flags = (0 if w is None else 1) | (2 if getattr(g, "symmetric", False) else 0)
        f.write(np.array([g.n, g.m, flags, src.size], dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(rp, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(col, dtype=np.int32).tobytes())
        if w is not None:
            f.write(np.ascontiguousarray(w, dtype=np.uint32).tobytes())
        f.write(src.tobytes())


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="write a named workload as a binary CSR file")
    ap.add_argument("workload")
    ap.add_argument("out")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--device", default="cuda")
    args = ap.parse_args(argv)
    import torch
    dev = torch.device(args.device if (args.device == "cpu" or torch.cuda.is_available()) else "cpu")
    g = make_workload(args.workload, dev, args.sources)
    write_csr(args.out, g)
    print(f"wrote {args.out}: {g.name} n={g.n} m={g.m} sources={len(g.sources or [])}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
