"""Invariant validator for BFS levels / SSSP distances and parent trees.

TEST INFRASTRUCTURE.  With every weight >= 1 the four checks below hold for
exactly one distance vector, the true shortest-path distances from ``src``,
so they pin full-size GPU results where the serial oracle would be slow:

 (i)   d[src] == 0 (and parent[src] == src);
 (ii)  for every edge (u, v, w) with d[u] finite: d[v] finite and
       d[v] <= d[u] + w                      (so d <= true distance);
 (iii) every reached v != src has a tight in-edge (p, v, w) with
       d[p] + w == d[v]; with parents given, p == parent[v]
                                             (so d >= true distance, because
                                              d strictly decreases along tight
                                              edges and only src has d == 0);
 (iv)  d[v] == INF  <=>  parent[v] == -1.

BFS levels are the unit-weight case.
"""
import numpy as np

INF = np.uint64(0xFFFFFFFF)


class ValidationError(AssertionError):
    pass


def validate(row_ptr, col, src: int, d, parent=None, w=None) -> None:
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    n = rp.size - 1
    dd = np.asarray(d).astype(np.uint32).astype(np.uint64)
    if dd.size != n:
        raise ValidationError(f"distance array has {dd.size} entries, expected {n}")
    ww = np.ones(c.size, dtype=np.uint64) if w is None else \
        np.asarray(w).astype(np.uint32).astype(np.uint64)
    if not (0 <= src < n):
        raise ValidationError("source out of range")
    # (i)
    if dd[src] != 0:
        raise ValidationError(f"d[src] = {int(dd[src])}, expected 0")
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    du = dd[u]
    dv = dd[c]
    fin_u = du != INF
    cand = du + ww
    # (ii)
    bad = fin_u & ((dv == INF) | (dv > cand))
    if bad.any():
        e = int(np.flatnonzero(bad)[0])
        raise ValidationError(
            f"edge {int(u[e])}->{int(c[e])} w={int(ww[e])}: d[u]={int(du[e])} d[v]={int(dv[e])} "
            "violates d[v] <= d[u] + w")
    tight = fin_u & (cand == dv)
    reached = dd != INF
    others = reached.copy()
    others[src] = False
    if parent is not None:
        p = np.asarray(parent).astype(np.int64)
        if p[src] != src:
            raise ValidationError(f"parent[src] = {int(p[src])}, expected src")
        # (iv)
        mism = reached != (p != -1)
        if mism.any():
            v = int(np.flatnonzero(mism)[0])
            raise ValidationError(f"vertex {v}: d={int(dd[v])} but parent={int(p[v])}")
        pr = p[others]
        if ((pr < 0) | (pr >= n)).any():
            raise ValidationError("parent out of range")
        tight = tight & (u == p[c])
    has_tight = np.zeros(n, dtype=bool)
    has_tight[c[tight]] = True
    # (iii)
    miss = others & ~has_tight
    if miss.any():
        v = int(np.flatnonzero(miss)[0])
        what = "parent edge" if parent is not None else "tight in-edge"
        raise ValidationError(f"vertex {v} (d={int(dd[v])}) has no {what}")
