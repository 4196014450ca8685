"""Pins of the minimum-spanning-forest oracle (the Boruvka workload of the
Atomic construct, Section 3) against facts fixed by mathematics or by an
independent library, not by the oracle itself:

* brute force over every edge subset of tiny connected graphs (the minimum
  spanning tree; with distinct weights it is unique, so edge sets match);
* scipy's minimum_spanning_tree weights on medium random graphs, connected or
  not (the forest weight is unique even when edges tie);
* closed forms: a path (every edge), a cycle with distinct weights (all but
  its heaviest edge), a star, a unit-weight grid (n - 1), a forest of
  disjoint triangles;
* the forest validator (cycle property + spanning) accepts the oracle's
  forest and rejects planted mistakes in it.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import minimum_spanning_tree

import oracle
from paper_1607_05707_amd import graphgen as gg


def _undirected(g):
    rp, c, w = g.numpy()
    src = np.repeat(np.arange(g.n), np.diff(rp))
    keep = src < c
    return src[keep], c[keep], w[keep].astype(np.int64)


def _forest_edges(g, in_forest):
    rp, c, w = g.numpy()
    src = np.repeat(np.arange(g.n), np.diff(rp))
    sel = (in_forest != 0) & (src < c)
    return sorted(zip(src[sel].tolist(), c[sel].tolist()))


def _sym(n, edges, name):
    """Undirected graph from (u, v, w) triples, both directions stored."""
    src = [u for u, v, _ in edges] + [v for u, v, _ in edges]
    dst = [v for u, v, _ in edges] + [u for u, v, _ in edges]
    ww = [x for _, _, x in edges] * 2
    return gg.from_edges(n, src, dst, ww, name=name)


def test_brute_force_on_tiny_connected_graphs():
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(200):
        n = int(rng.integers(2, 7))
        pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
        k = int(rng.integers(n - 1, len(pairs) + 1))
        chosen = [pairs[i] for i in rng.choice(len(pairs), size=k, replace=False)]
        distinct = trial % 2 == 0
        ws = rng.permutation(np.arange(1, k + 1)) if distinct else rng.integers(1, 4, size=k)
        edges = [(u, v, int(x)) for (u, v), x in zip(chosen, ws)]
        g = _sym(n, edges, f"tiny{trial}")
        weight, in_forest, comp, ne = oracle.kruskal(*g.numpy())
        best, best_sets = None, []
        for sub in itertools.combinations(range(k), n - 1):
            parent = list(range(n))

            def find(x):
                while parent[x] != x:
                    x = parent[x]
                return x
            ok = True
            for i in sub:
                a, b = find(edges[i][0]), find(edges[i][1])
                if a == b:
                    ok = False
                    break
                parent[a] = b
            if not ok:
                continue
            tot = sum(edges[i][2] for i in sub)
            if best is None or tot < best:
                best, best_sets = tot, [sub]
            elif tot == best:
                best_sets.append(sub)
        if best is None:  # the random graph is disconnected
            continue
        checked += 1
        assert weight == best and ne == n - 1
        assert set(comp.tolist()) == {0}
        if distinct:
            assert len(best_sets) == 1
            want = sorted((min(edges[i][0], edges[i][1]), max(edges[i][0], edges[i][1])) for i in best_sets[0])
            assert _forest_edges(g, in_forest) == want
        assert oracle.validate_forest(*g.numpy(), in_forest) == weight
    assert checked > 100


@pytest.mark.parametrize("maker", [
    lambda: gg.rmat(10, seed=3, weight_seed=4, wmax=255),
    lambda: gg.uniform_random(1500, 3.0, seed=5, weight_seed=6, wmax=1000),
    lambda: gg.uniform_random(800, 0.7, seed=7, weight_seed=8, wmax=9),
    lambda: gg.config_road(width=40),
])
def test_weight_matches_scipy(maker):
    g = maker()
    rp, c, w = g.numpy()
    weight, in_forest, comp, ne = oracle.kruskal(rp, c, w)
    m = sp.csr_matrix((w.astype(np.float64), c, rp), shape=(g.n, g.n))
    assert weight == int(round(minimum_spanning_tree(m).sum()))
    ncomp = sp.csgraph.connected_components(m, directed=False)[0]
    assert ne == g.n - ncomp
    assert len(set(comp.tolist())) == ncomp
    assert all(comp[v] <= v for v in range(g.n))
    if g.n <= 2000:
        assert oracle.validate_forest(rp, c, w, in_forest) == weight


def test_closed_forms():
    n = 50
    path = _sym(n, [(i, i + 1, 3 + i % 5) for i in range(n - 1)], "path")
    weight, in_forest, _, ne = oracle.kruskal(*path.numpy())
    assert ne == n - 1 and weight == sum(3 + i % 5 for i in range(n - 1)) and in_forest.all()
    cyc = [(i, (i + 1) % n, 10 + i) for i in range(n)]
    weight, in_forest, _, ne = oracle.kruskal(*_sym(n, cyc, "cycle").numpy())
    assert ne == n - 1 and weight == sum(10 + i for i in range(n)) - (10 + n - 1)
    star = _sym(n, [(0, i, i) for i in range(1, n)], "star")
    weight, _, _, ne = oracle.kruskal(*star.numpy())
    assert ne == n - 1 and weight == sum(range(1, n))
    grid = gg.grid2d(17, 13, weight_seed=1, wmax=1)
    weight, _, comp, ne = oracle.kruskal(*grid.numpy())
    assert weight == ne == grid.n - 1 and set(comp.tolist()) == {0}
    tri = _sym(30, [e for t in range(10) for e in ((3 * t, 3 * t + 1, 5), (3 * t + 1, 3 * t + 2, 7),
                                                    (3 * t, 3 * t + 2, 6))], "triangles")
    weight, _, comp, ne = oracle.kruskal(*tri.numpy())
    assert ne == 20 and weight == 10 * (5 + 6)
    assert sorted(set(comp.tolist())) == [3 * t for t in range(10)]
    one = gg.from_edges(1, [], [], [], name="single")
    assert oracle.kruskal(*one.numpy())[0] == 0


def test_validator_rejects_planted_mistakes():
    g = gg.uniform_random(300, 4.0, seed=11, weight_seed=12, wmax=100)
    rp, c, w = g.numpy()
    weight, in_forest, _, _ = oracle.kruskal(rp, c, w)
    assert oracle.validate_forest(rp, c, w, in_forest) == weight
    src = np.repeat(np.arange(g.n), np.diff(rp))

    def rev(e):
        return next(f for f in range(rp[c[e]], rp[c[e] + 1]) if c[f] == src[e])

    tree = [e for e in np.nonzero(in_forest)[0] if src[e] < c[e]]
    other = [e for e in range(c.size) if not in_forest[e] and src[e] < c[e]]
    # a dropped forest edge: one tree too many
    bad = in_forest.copy()
    bad[tree[0]] = bad[rev(tree[0])] = 0
    with pytest.raises(oracle.ValidationError):
        oracle.validate_forest(rp, c, w, bad)
    # an extra edge closes a cycle
    bad = in_forest.copy()
    bad[other[0]] = bad[rev(other[0])] = 1
    with pytest.raises(oracle.ValidationError):
        oracle.validate_forest(rp, c, w, bad)
    # one direction only
    bad = in_forest.copy()
    bad[rev(tree[1])] = 0
    with pytest.raises(oracle.ValidationError):
        oracle.validate_forest(rp, c, w, bad)
    # a heavier spanning forest: swap a forest edge for a non-forest edge on its cut
    swapped = False
    for e in other:
        bad = in_forest.copy()
        bad[e] = bad[rev(e)] = 1
        # drop the heaviest forest edge on the cycle that e closes, if any is lighter than e
        for t in sorted(tree, key=lambda t: (-int(w[t]), -int(src[t]), -int(c[t]))):
            if (int(w[t]), int(src[t]), int(c[t])) >= (int(w[e]), int(src[e]), int(c[e])):
                continue
            trial = bad.copy()
            trial[t] = trial[rev(t)] = 0
            try:
                oracle.validate_forest(rp, c, w, trial)
            except oracle.ValidationError as err:
                if "closes a cycle" in str(err) or "trees" in str(err):
                    continue
                swapped = True
                break
            raise AssertionError("a heavier spanning forest was accepted")
        if swapped:
            break
    assert swapped


def test_asymmetric_input_is_rejected():
    g = gg.from_edges(3, [0, 1], [1, 2], [4, 5], name="directed")
    with pytest.raises(ValueError):
        oracle.kruskal(*g.numpy())


def test_asymmetric_weights_and_one_sided_reverse_are_rejected():
    # 0-1 stored both ways but with different weights
    rp = np.array([0, 1, 2], dtype=np.int32)
    c = np.array([1, 0], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.kruskal(rp, c, np.array([3, 4], dtype=np.uint32))
    # only the u > v entry of an edge (the other half is empty)
    rp = np.array([0, 0, 1], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.kruskal(rp, np.array([0], dtype=np.int32), np.array([3], dtype=np.uint32))


def test_parallel_edges_take_the_lighter_copy():
    # 0-1 twice (weights 7 and 2, each stored both ways), 1-2 once (weight 5)
    rp = np.array([0, 2, 5, 6], dtype=np.int32)
    c = np.array([1, 1, 0, 0, 2, 1], dtype=np.int32)
    w = np.array([7, 2, 2, 7, 5, 5], dtype=np.uint32)
    weight, in_forest, comp, ne = oracle.kruskal(rp, c, w)
    assert (weight, ne) == (7, 2)
    assert in_forest.tolist() == [0, 1, 1, 0, 1, 1]
    assert comp.tolist() == [0, 0, 0]
