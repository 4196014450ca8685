"""Seeded synthetic meshes for Delaunay mesh refinement (inputs only).

The domain is the unit square.  Its boundary carries k evenly spaced points
per side (the corners included); the interior holds npoints points drawn
uniformly from a counter-based stream.  The input mesh is the Delaunay
triangulation of all of them (scipy's Qhull), stored in the library's
layout: points float64[P, 2]; triangles int32[T, 4] = (v0, v1, v2, live
flag), counter-clockwise; neighbours int32[T, 4] where entry i is the
triangle across edge (v_i, v_(i+1) mod 3) and -1 marks the domain boundary.
Arrays are sized to a capacity (rows beyond the input are zero: dead
triangles, unused points) so that refinement can append in place.

This module holds no refinement arithmetic; it only builds inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .graphgen import rand_u32

_S_MESH_X = 0x4D455358
_S_MESH_Y = 0x4D455359


@dataclass
class Mesh:
    pts: np.ndarray      # float64[P_cap, 2]
    tri: np.ndarray      # int32[T_cap, 4]
    nbr: np.ndarray      # int32[T_cap, 4]
    npts: int            # points in use
    ntri: int            # triangle slots in use
    name: str

    @property
    def input_pts(self) -> np.ndarray:
        return self.pts[:self.npts].copy()


def _uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles in (0, 1) from the counter-based generator (53 bits from two
    32-bit words)."""
    idx = torch.arange(2 * n, dtype=torch.int64)
    w = rand_u32(seed, stream, idx).numpy().astype(np.uint64)
    hi = w[0::2] >> np.uint64(5)   # 27 bits
    lo = w[1::2] >> np.uint64(6)   # 26 bits
    x = (hi.astype(np.float64) * 67108864.0 + lo.astype(np.float64) + 0.5) / 9007199254740992.0
    return x


def random_square(npoints: int, seed: int, k: int = 0, tri_factor: float = 8.0, pt_factor: float = 6.0) -> Mesh:
    """Delaunay mesh of npoints uniform points in the unit square plus k
    evenly spaced points per side (default about sqrt(npoints) / 2)."""
    from scipy.spatial import Delaunay
    k = k or max(4, int(round(math.sqrt(npoints) / 2)))
    s = np.arange(k, dtype=np.float64) / k
    z, o = np.zeros(k), np.ones(k)
    boundary = np.concatenate([np.stack([s, z], 1), np.stack([o, s], 1), np.stack([1.0 - s, o], 1),
                               np.stack([z, 1.0 - s], 1)])
    inner = np.stack([_uniform01(seed, _S_MESH_X, npoints), _uniform01(seed, _S_MESH_Y, npoints)], 1)
    pts = np.concatenate([boundary, inner])
    d = Delaunay(pts)
    t = d.simplices.astype(np.int64)
    # scipy's neighbour j is opposite vertex j; entry i here is across edge (v_i, v_i+1)
    nb = d.neighbors.astype(np.int64)[:, [2, 0, 1]]
    a = pts[t]
    det = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    cw = det < 0
    t[cw] = t[cw][:, [0, 2, 1]]
    nb[cw] = nb[cw][:, [2, 1, 0]]
    T = t.shape[0]
    tcap = max(16, int(T * tri_factor))
    pcap = max(16, int(pts.shape[0] * pt_factor))
    P = np.zeros((pcap, 2), dtype=np.float64)
    P[:pts.shape[0]] = pts
    tri = np.zeros((tcap, 4), dtype=np.int32)
    tri[:T, :3] = t
    tri[:T, 3] = 1
    nbr = np.full((tcap, 4), -1, dtype=np.int32)
    nbr[:T, :3] = nb
    return Mesh(P, tri, nbr, pts.shape[0], T, f"square_n{npoints}_k{k}_s{seed}")


MAGIC = b"IRGLMSH1"


def write_mesh(path: str, m: Mesh) -> None:
    """Binary mesh file for the native runner (little endian): b"IRGLMSH1",
    int64 npts, ntri, pcap, tcap, float64 pts[pcap][2], int32 tri[tcap][4],
    int32 nbr[tcap][4]."""
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(np.array([m.npts, m.ntri, m.pts.shape[0], m.tri.shape[0]], dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(m.pts, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(m.tri, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(m.nbr, dtype=np.int32).tobytes())


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="write a random-square mesh as a binary file")
    ap.add_argument("out")
    ap.add_argument("--points", type=int, default=1000000)
    ap.add_argument("--seed", type=int, default=42)
    args = ap.parse_args(argv)
    m = random_square(args.points, args.seed)
    write_mesh(args.out, m)
    print(f"wrote {args.out}: {m.name} points={m.npts} triangles={m.ntri}", flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
