"""Floyd-Warshall all-pairs shortest paths (numpy, int64) for tiny graphs.

TEST INFRASTRUCTURE: an independent check of the serial oracle.  Textbook
min-plus closure: D_k[i,j] = min(D_{k-1}[i,j], D_{k-1}[i,k] + D_{k-1}[k,j]).
"""
import numpy as np

BIG = np.int64(1) << 60


def floyd_warshall(n: int, row_ptr, col, w=None) -> np.ndarray:
    """Return D (int64 [n,n]); D[i,j] = BIG when j is unreachable from i.
    ``w=None`` means unit weights (hop counts).  Parallel edges keep the
    smallest weight; self-loops never shorten a path (weights >= 1)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    ww = np.ones(c.size, dtype=np.int64) if w is None else np.asarray(w).astype(np.uint32).astype(np.int64)
    d = np.full((n, n), BIG, dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(rp))
    np.minimum.at(d, (src, c), ww)
    d[np.arange(n), np.arange(n)] = 0
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
        d = np.minimum(d, BIG)
    return d
