"""Pins of the CPU oracle against facts fixed by mathematics, not by itself.

* Floyd-Warshall all-pairs closure on hundreds of tiny random graphs
  (directed, undirected, self-loops, multi-edges, disconnected);
* scipy's library shortest-path routines on medium graphs;
* closed forms: grid Manhattan distance, path, directed cycle, star,
  complete graph, random tree path sums, uniform weight c -> c * level;
* validator mutation tests (a planted mistake in an oracle output must be
  rejected), overflow detection.

The paper prints no worked example with values, so there is no golden
fixture from it; see tests/golden/README.md.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_1607_05707_amd import graphgen as gg

INF = oracle.INF


def _fw_row(g, src, weighted):
    rp, c, w = g.numpy()
    d = oracle.floyd_warshall(g.n, rp, c, w if weighted else None)[src]
    out = np.full(g.n, INF, dtype=np.uint64)
    fin = d < oracle.fw.BIG
    out[fin] = d[fin]
    return out.astype(np.uint32)


def _tiny_graphs():
    rng = np.random.default_rng(12345)
    for i in range(320):
        n = int(rng.integers(1, 41))
        kind = i % 4
        if kind == 0:      # directed, self-loops and multi-edges kept
            m = int(rng.integers(0, 4 * n + 1))
            g = gg.random_directed(n, m, seed=i, weight_seed=1000 + i, wmax=20)
        elif kind == 1:    # undirected, simple
            g = gg.uniform_random(n, float(rng.uniform(0.5, 6.0)), seed=i, weight_seed=2000 + i, wmax=50)
        elif kind == 2:    # sparse directed: many unreachable vertices
            g = gg.random_directed(n, max(0, n // 2), seed=i, weight_seed=3000 + i, wmax=5)
        else:              # dense directed with large weights
            g = gg.random_directed(n, n * n, seed=i, weight_seed=4000 + i, wmax=1 << 20)
        src = int(rng.integers(0, n))
        yield g, src


def test_oracle_matches_floyd_warshall_on_tiny_graphs(oracle_lib):
    count = 0
    for g, src in _tiny_graphs():
        rp, c, w = g.numpy()
        lv, pl = oracle.bfs(rp, c, src)
        np.testing.assert_array_equal(lv, _fw_row(g, src, weighted=False), err_msg=g.name)
        dist, pd = oracle.dijkstra(rp, c, w, src)
        np.testing.assert_array_equal(dist, _fw_row(g, src, weighted=True), err_msg=g.name)
        oracle.validate(rp, c, src, lv, pl)
        oracle.validate(rp, c, src, dist, pd, w)
        count += 1
    assert count == 320


def _scipy_dist(g, src, weighted):
    rp, c, w = g.numpy()
    # scipy would sum parallel edges: keep the lightest of each (u, v) pair
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    key = u * g.n + c
    ukey, first = np.unique(key, return_index=True)
    wt = w.astype(np.float64) if weighted else np.ones(c.size)
    data = np.minimum.reduceat(wt, first) if c.size else wt
    mat = sp.csr_matrix((data, (ukey // g.n, ukey % g.n)), shape=(g.n, g.n))
    d = shortest_path(mat, method="D", directed=True, unweighted=not weighted, indices=src)
    out = np.full(g.n, INF, dtype=np.uint64)
    fin = np.isfinite(d)
    out[fin] = d[fin].astype(np.uint64)
    return out.astype(np.uint32)


@pytest.mark.parametrize("maker", [
    lambda: gg.uniform_random(3000, 5.0, seed=11, weight_seed=12, wmax=1000),
    lambda: gg.rmat(11, seed=13, weight_seed=14, wmax=255),
    lambda: gg.grid2d(40, weight_seed=15, wmax=10000, drop_p=0.05, long_frac=0.01, seed=16),
    lambda: gg.random_directed(2000, 6000, seed=17, weight_seed=18, wmax=100),
])
def test_oracle_matches_scipy(oracle_lib, maker):
    g = maker()
    rp, c, w = g.numpy()
    for src in gg.pick_sources(g, 5, seed=99):
        lv, _ = oracle.bfs(rp, c, src)
        np.testing.assert_array_equal(lv, _scipy_dist(g, src, weighted=False))
        dist, _ = oracle.dijkstra(rp, c, w, src)
        np.testing.assert_array_equal(dist, _scipy_dist(g, src, weighted=True))


def test_grid_manhattan_closed_form(oracle_lib):
    W, H = 37, 23
    g = gg.grid2d(W, H)
    rp, c, _ = g.numpy()
    ids = np.arange(W * H)
    r, cc = ids // W, ids % W
    for src in [0, W * H - 1, 11 * W + 17, W - 1]:
        lv, p = oracle.bfs(rp, c, src)
        sr, sc = src // W, src % W
        np.testing.assert_array_equal(lv, (np.abs(r - sr) + np.abs(cc - sc)).astype(np.uint32))
        oracle.validate(rp, c, src, lv, p)
    g64 = gg.config_grid64()
    lv, _ = oracle.bfs(*g64.numpy()[:2], 0)
    assert int(lv.max()) == 126
    hist = oracle.level_histogram(lv)
    expected = [min(k + 1, 127 - k, 64) for k in range(127)]
    np.testing.assert_array_equal(hist, expected)


def test_path_graphs(oracle_lib):
    n = 200
    rng = np.random.default_rng(3)
    wts = rng.integers(1, 1000, n - 1)
    # undirected weighted path 0 - 1 - ... - n-1
    src = list(range(n - 1)) + list(range(1, n))
    dst = list(range(1, n)) + list(range(n - 1))
    w = list(wts) + list(wts)
    g = gg.from_edges(n, src, dst, w)
    rp, c, ww = g.numpy()
    prefix = np.concatenate([[0], np.cumsum(wts)])
    for s in [0, 57, n - 1]:
        lv, _ = oracle.bfs(rp, c, s)
        np.testing.assert_array_equal(lv, np.abs(np.arange(n) - s).astype(np.uint32))
        d, p = oracle.dijkstra(rp, c, ww, s)
        np.testing.assert_array_equal(d, np.abs(prefix - prefix[s]).astype(np.uint32))
        oracle.validate(rp, c, s, d, p, ww)
    # directed path: only forward reachable
    gd = gg.from_edges(n, range(n - 1), range(1, n), wts)
    lv, _ = oracle.bfs(*gd.numpy()[:2], 50)
    exp = np.where(np.arange(n) >= 50, np.arange(n) - 50, INF).astype(np.uint32)
    np.testing.assert_array_equal(lv, exp)


def test_directed_cycle(oracle_lib):
    n = 97
    g = gg.from_edges(n, range(n), [(i + 1) % n for i in range(n)], [3] * n)
    rp, c, w = g.numpy()
    for s in [0, 40]:
        lv, _ = oracle.bfs(rp, c, s)
        np.testing.assert_array_equal(lv, ((np.arange(n) - s) % n).astype(np.uint32))
        d, _ = oracle.dijkstra(rp, c, w, s)
        np.testing.assert_array_equal(d, (3 * ((np.arange(n) - s) % n)).astype(np.uint32))


def test_star_and_complete(oracle_lib):
    n = 500
    src = [0] * (n - 1) + list(range(1, n))
    dst = list(range(1, n)) + [0] * (n - 1)
    g = gg.from_edges(n, src, dst)
    rp, c, _ = g.numpy()
    lv, _ = oracle.bfs(rp, c, 0)
    np.testing.assert_array_equal(lv, np.array([0] + [1] * (n - 1), dtype=np.uint32))
    lv, _ = oracle.bfs(rp, c, 7)
    exp = np.full(n, 2, dtype=np.uint32)
    exp[0] = 1
    exp[7] = 0
    np.testing.assert_array_equal(lv, exp)
    k = 30
    pairs = [(i, j) for i in range(k) for j in range(k) if i != j]
    gc = gg.from_edges(k, [a for a, _ in pairs], [b for _, b in pairs])
    lv, _ = oracle.bfs(*gc.numpy()[:2], 4)
    exp = np.ones(k, dtype=np.uint32)
    exp[4] = 0
    np.testing.assert_array_equal(lv, exp)


def test_random_tree_path_sums(oracle_lib):
    rng = np.random.default_rng(8)
    n = 3000
    par = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)])
    wt = rng.integers(1, 10 ** 6, n)
    src = []
    dst = []
    w = []
    for v in range(1, n):
        src += [par[v], v]
        dst += [v, par[v]]
        w += [wt[v], wt[v]]
    g = gg.from_edges(n, src, dst, w)
    rp, c, ww = g.numpy()
    # root distances by walking parent pointers (independent of any search)
    depth = np.zeros(n, dtype=np.int64)
    rootd = np.zeros(n, dtype=np.int64)
    for v in range(1, n):
        depth[v] = depth[par[v]] + 1
        rootd[v] = rootd[par[v]] + wt[v]
    lv, _ = oracle.bfs(rp, c, 0)
    np.testing.assert_array_equal(lv, depth.astype(np.uint32))
    d, p = oracle.dijkstra(rp, c, ww, 0)
    np.testing.assert_array_equal(d, rootd.astype(np.uint32))
    np.testing.assert_array_equal(p[1:], par[1:])


def test_uniform_weight_is_scaled_level(oracle_lib):
    g = gg.rmat(12, seed=21)
    rp, c, _ = g.numpy()
    for cst in [1, 7, 1000]:
        w = np.full(c.size, cst, dtype=np.uint32)
        s = gg.pick_sources(g, 1, seed=cst)[0]
        lv, _ = oracle.bfs(rp, c, s)
        d, _ = oracle.dijkstra(rp, c, w, s)
        exp = np.where(lv == INF, np.uint64(INF), lv.astype(np.uint64) * cst).astype(np.uint32)
        np.testing.assert_array_equal(d, exp)


def test_histogram(oracle_lib):
    g = gg.rmat(12, seed=5)
    rp, c, _ = g.numpy()
    s = gg.pick_sources(g, 1, seed=1)[0]
    lv, _ = oracle.bfs(rp, c, s)
    hist = oracle.level_histogram(lv)
    assert hist[0] == 1 and hist.sum() == int((lv != INF).sum())


def test_edges_scanned_closed_forms(oracle_lib):
    # Every value below is fixed by the graph's shape alone (counted by hand
    # or by a closed form), not by re-evaluating the oracle's own formula.
    # (a) a connected symmetric graph: every vertex is reached from any
    #     source, so every one of its m CSR entries is scanned
    g64 = gg.config_grid64()
    rp, c, _ = g64.numpy()
    assert g64.m == 2 * 2 * 64 * 63 == 16128
    for s in (0, 1234, 4095):
        lv, _ = oracle.bfs(rp, c, s)
        assert oracle.edges_scanned(rp, lv) == 16128
    # (b) directed path 0 -> 1 -> ... -> n-1 from s: vertices s..n-1 are
    #     reached and all but the last have one out-edge
    n = 300
    gp = gg.from_edges(n, range(n - 1), range(1, n))
    for s in (0, 17, n - 2, n - 1):
        lv, _ = oracle.bfs(*gp.numpy()[:2], s)
        assert oracle.edges_scanned(gp.numpy()[0], lv) == n - 1 - s
    # (c) an unreachable part: a symmetric star on 0..5 (10 entries), a
    #     triangle 6, 7, 8 (6 entries) and an isolated vertex 9; from the star
    #     centre 10 entries, from a triangle corner 6, from 9 none
    src = [0, 0, 0, 0, 0, 1, 2, 3, 4, 5, 6, 7, 7, 8, 8, 6]
    dst = [1, 2, 3, 4, 5, 0, 0, 0, 0, 0, 7, 6, 8, 7, 6, 8]
    gs = gg.from_edges(10, src, dst)
    rps, cs, _ = gs.numpy()
    for s, want in ((0, 10), (3, 10), (7, 6), (9, 0)):
        lv, _ = oracle.bfs(rps, cs, s)
        assert oracle.edges_scanned(rps, lv) == want, (s, want)
    # (d) directed cycle of n: all n entries from any source
    gc = gg.from_edges(97, range(97), [(i + 1) % 97 for i in range(97)])
    lv, _ = oracle.bfs(*gc.numpy()[:2], 40)
    assert oracle.edges_scanned(gc.numpy()[0], lv) == 97
    # (e) a directed out-star 0 -> 1..k plus edges 1 -> 0 back: from leaf 1
    #     everything is reached (k + 1 entries); from leaf 2, which has no
    #     out-edge, only 2 itself (0 entries)
    k = 50
    go = gg.from_edges(k + 1, [0] * k + [1], list(range(1, k + 1)) + [0])
    rpo, co, _ = go.numpy()
    lv, _ = oracle.bfs(rpo, co, 1)
    assert oracle.edges_scanned(rpo, lv) == k + 1
    lv, _ = oracle.bfs(rpo, co, 2)
    assert oracle.edges_scanned(rpo, lv) == 0


def test_certificate_accepts_exact_and_rejects_planted_mistakes(oracle_lib):
    # accepted: the Floyd-Warshall distances of tiny graphs (independent of
    # Dijkstra) and of medium graphs checked against scipy above
    checked = 0
    for g, src in _tiny_graphs():
        rp, c, w = g.numpy()
        oracle.certify(rp, c, src, _fw_row(g, src, weighted=True), w)
        oracle.certify(rp, c, src, _fw_row(g, src, weighted=False))
        checked += 1
    assert checked == 320
    g = gg.uniform_random(3000, 6.0, seed=41, weight_seed=42, wmax=100)
    rp, c, w = g.numpy()
    s = gg.pick_sources(g, 1, seed=4)[0]
    d = _scipy_dist(g, s, weighted=True)
    lv = _scipy_dist(g, s, weighted=False)
    oracle.certify(rp, c, s, d, w)
    oracle.certify(rp, c, s, lv)
    reached = np.flatnonzero((d != INF) & (np.arange(g.n) != s))
    rng = np.random.default_rng(5)
    for v in rng.choice(reached, 20, replace=False):
        for delta in (-1, 1):
            bad = d.copy()
            bad[v] = np.uint32(int(bad[v]) + delta)
            with pytest.raises(oracle.ValidationError):
                oracle.certify(rp, c, s, bad, w)
            badl = lv.copy()
            badl[v] = np.uint32(int(badl[v]) + delta)
            with pytest.raises(oracle.ValidationError):
                oracle.certify(rp, c, s, badl)
        bad = d.copy()
        bad[v] = INF
        with pytest.raises(oracle.ValidationError):
            oracle.certify(rp, c, s, bad, w)
    # a distance for a vertex that cannot be reached, and a wrong source value
    gd = gg.from_edges(4, [0, 1], [1, 2], [5, 5])
    rpd, cd, wd = gd.numpy()
    oracle.certify(rpd, cd, 0, np.array([0, 5, 10, INF], dtype=np.uint32), wd)
    with pytest.raises(oracle.ValidationError):
        oracle.certify(rpd, cd, 0, np.array([0, 5, 10, 3], dtype=np.uint32), wd)
    with pytest.raises(oracle.ValidationError):
        oracle.certify(rpd, cd, 0, np.array([1, 5, 10, INF], dtype=np.uint32), wd)
    # a whole vector shifted by one everywhere except the source has no tight edge
    with pytest.raises(oracle.ValidationError):
        oracle.certify(rpd, cd, 0, np.array([0, 4, 9, INF], dtype=np.uint32), wd)


def test_validator_rejects_planted_mistakes(oracle_lib):
    g = gg.uniform_random(2000, 6.0, seed=31, weight_seed=32, wmax=100)
    rp, c, w = g.numpy()
    s = gg.pick_sources(g, 1, seed=3)[0]
    d, p = oracle.dijkstra(rp, c, w, s)
    lv, pl = oracle.bfs(rp, c, s)
    oracle.validate(rp, c, s, d, p, w)
    oracle.validate(rp, c, s, d, None, w)
    reached = np.flatnonzero((d != INF) & (np.arange(g.n) != s))
    rng = np.random.default_rng(0)
    for v in rng.choice(reached, 10, replace=False):
        for delta in (-1, 1):
            bad = d.copy()
            bad[v] = np.uint32(int(bad[v]) + delta)
            with pytest.raises(oracle.ValidationError):
                oracle.validate(rp, c, s, bad, None, w)
        badl = lv.copy()
        badl[v] = np.uint32(int(badl[v]) + 1)
        with pytest.raises(oracle.ValidationError):
            oracle.validate(rp, c, s, badl, None)
        # a parent that is a neighbour but not tight
        nbrs = c[rp[v]:rp[v + 1]]
        loose = [u for u in nbrs if d[u] != INF and int(d[u]) + int(w[rp[u]:rp[u + 1]][np.searchsorted(
            c[rp[u]:rp[u + 1]], v)]) != int(d[v])]
        if loose:
            bp = p.copy()
            bp[v] = loose[0]
            with pytest.raises(oracle.ValidationError):
                oracle.validate(rp, c, s, d, bp, w)
    # flip a reached vertex to INF / an unreached one to finite
    bad = d.copy()
    bad[reached[0]] = INF
    with pytest.raises(oracle.ValidationError):
        oracle.validate(rp, c, s, bad, None, w)
    bad = d.copy()
    bad[s] = 1
    with pytest.raises(oracle.ValidationError):
        oracle.validate(rp, c, s, bad, None, w)


def test_dijkstra_overflow_detected(oracle_lib):
    n = 4
    g = gg.from_edges(n, [0, 1, 2], [1, 2, 3], [0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF])
    rp, c, w = g.numpy()
    with pytest.raises(OverflowError):
        oracle.dijkstra(rp, c, w, 0)
    d, _ = oracle.dijkstra(rp, c, w, 1)   # 1 -> 2 -> 3: 2^32 - 2 fits
    assert int(d[3]) == 0xFFFFFFFE


def test_unreachable_and_single_vertex(oracle_lib):
    g = gg.from_edges(1, [], [])
    lv, p = oracle.bfs(*g.numpy()[:2], 0)
    assert lv.tolist() == [0] and p.tolist() == [0]
    g = gg.from_edges(5, [0, 1], [1, 0])
    lv, p = oracle.bfs(*g.numpy()[:2], 0)
    assert lv.tolist() == [0, 1, INF, INF, INF]
    assert p.tolist() == [0, 0, -1, -1, -1]
