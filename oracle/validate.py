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


def validate_forest(row_ptr, col, w, in_forest) -> int:
    """Check that ``in_forest`` (uint8 per CSR entry) marks the minimum
    spanning forest of the symmetric CSR under the total edge order (w, u, v),
    independently of how it was computed, and return its weight:

     (i)   every marked entry's reverse is marked (the forest is undirected);
     (ii)  the marked edges form a forest (no cycle) that connects exactly the
           vertex sets of the graph's connected components;
     (iii) cycle property: every unmarked edge {u, v} is larger, in the total
           order, than each forest edge on the forest path from u to v.

    (ii) and (iii) characterize the minimum spanning forest; under a total
    order it is unique.  Plain Python loops: small graphs only."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    ww = np.asarray(w, dtype=np.int64)
    f = np.asarray(in_forest, dtype=np.uint8)
    n = rp.size - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    key = {}
    for e in range(c.size):
        u, v = int(src[e]), int(c[e])
        key[e] = (int(ww[e]), min(u, v), max(u, v))
    # (i) symmetric marks
    marked = {}
    for e in np.nonzero(f)[0]:
        u, v = int(src[e]), int(c[e])
        if u == v:
            raise ValidationError(f"self-loop {u} in the forest")
        marked[(min(u, v), max(u, v))] = key[int(e)]
    for e in np.nonzero(f)[0]:
        u, v = int(src[e]), int(c[e])
        back = [g for g in range(rp[v], rp[v + 1]) if int(c[g]) == u and f[g]]
        if not back:
            raise ValidationError(f"forest edge {u}->{v} lacks its marked reverse")
    # (ii) forest: union-find over marked edges must never close a cycle
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for (u, v) in marked:
        a, b = find(u), find(v)
        if a == b:
            raise ValidationError(f"forest edge {{{u}, {v}}} closes a cycle")
        parent[a] = b
    gparent = list(range(n))

    def gfind(x):
        while gparent[x] != x:
            gparent[x] = gparent[gparent[x]]
            x = gparent[x]
        return x

    for e in range(c.size):
        a, b = gfind(int(src[e])), gfind(int(c[e]))
        if a != b:
            gparent[a] = b
    # forest edges are graph edges, so forest trees refine graph components:
    # equal counts mean equal vertex sets
    roots_f = {find(v) for v in range(n)}
    roots_g = {gfind(v) for v in range(n)}
    if len(roots_f) != len(roots_g):
        raise ValidationError(f"forest has {len(roots_f)} trees, the graph {len(roots_g)} components")
    # (iii) cycle property over a rooted forest
    adj = [[] for _ in range(n)]
    for (u, v), k in marked.items():
        adj[u].append((v, k))
        adj[v].append((u, k))
    up = [-1] * n
    upkey = [None] * n
    depth = [0] * n
    seen = [False] * n
    for r in range(n):
        if seen[r]:
            continue
        seen[r] = True
        stack = [r]
        while stack:
            x = stack.pop()
            for y, k in adj[x]:
                if not seen[y]:
                    seen[y] = True
                    up[y], upkey[y], depth[y] = x, k, depth[x] + 1
                    stack.append(y)
    for e in range(c.size):
        u, v = int(src[e]), int(c[e])
        if u >= v or (u, v) in marked:
            continue
        k = key[e]
        a, b, worst = u, v, None
        while a != b:
            if depth[a] < depth[b]:
                a, b = b, a
            if worst is None or upkey[a] > worst:
                worst = upkey[a]
            a = up[a]
        if worst is not None and worst > k:
            raise ValidationError(f"edge {{{u}, {v}}} {k} is smaller than forest edge {worst} on its cycle")
    return sum(k[0] for k in marked.values())
