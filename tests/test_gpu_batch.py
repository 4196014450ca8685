"""Batched launch: many BFS/SSSP queries of uneven size in one persistent
launch.  Every task must equal the oracle bit for bit and equal its own
single-query run; parents are validated by the invariants."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_05707_amd import graphgen as gg

pytestmark = pytest.mark.gpu

BFS, SSSP = 0, 1


@pytest.fixture(scope="module")
def irgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_05707_amd import irgl as mod
    return mod


@pytest.fixture(scope="module")
def graphs(irgl):
    dev = torch.device("cuda:0")
    gs = [gg.config_grid64(), gg.rmat(12, seed=3, weight_seed=4), gg.config_road(width=96),
          gg.uniform_random(5000, 6.0, seed=5, weight_seed=6, wmax=1000),
          gg.uniform_random(300, 3.0, seed=7, weight_seed=8, wmax=50),
          gg.random_directed(2000, 9000, seed=9, weight_seed=10, wmax=100)]
    out = []
    for g in gs:
        gd = g.to(dev)
        out.append((gd, irgl.upload(gd), g.numpy()))
    return out


def _ref(kind, np_g, src):
    rp, col, w = np_g
    return oracle.bfs(rp, col, src)[0] if kind == BFS else oracle.dijkstra(rp, col, w, src)[0]


def _make_tasks(irgl, graphs, per_graph, with_parent, seed):
    rng = np.random.default_rng(seed)
    tasks, meta = [], []
    for gi, (g, hg, np_g) in enumerate(graphs):
        srcs = gg.pick_sources(g, per_graph, seed=100 + gi)
        for j, s in enumerate(srcs):
            kind = int(rng.integers(0, 2))
            tasks.append(irgl.Task(hg, kind, s, with_parent=with_parent, tag=len(tasks)))
            meta.append((gi, kind, s))
    return tasks, meta


@pytest.mark.parametrize("team,block,barrier", [(16, 256, 0), (1, 256, 0), (4, 512, 0), (10_000, 256, 0),
                                                (16, 256, 1), (3, 256, 0), (10_000, 256, 1)])
def test_batch_matches_oracle(irgl, graphs, team, block, barrier):
    tasks, meta = _make_tasks(irgl, graphs, per_graph=5, with_parent=(team == 16), seed=team)
    print(f"[case] batch team={team} block={block} barrier={barrier} tasks={len(tasks)}", flush=True)
    b = irgl.irgl_batch_submit(tasks, cfg={"team": team, "block": block, "barrier": barrier})
    stats = irgl.irgl_batch_wait(b)
    for t, (gi, kind, s), st in zip(tasks, meta, stats):
        g, hg, np_g = graphs[gi]
        assert st["status"] == 0, (gi, kind, s, st)
        got = irgl.as_u32_numpy(t.out)
        ref = _ref(kind, np_g, s)
        np.testing.assert_array_equal(got, ref, err_msg=f"graph {gi} kind {kind} src {s}")
        if t.parent is not None:
            rp, col, w = np_g
            oracle.validate(rp, col, s, got, t.parent.cpu().numpy(), None if kind == BFS else w)
        if kind == BFS:
            assert st["iterations"] == int(ref[ref != oracle.INF].max()) + 1
            assert st["frontier_edges"] == oracle.edges_scanned(np_g[0], ref)
    b.free()


def test_batch_equals_single_queries(irgl, graphs):
    tasks, meta = _make_tasks(irgl, graphs, per_graph=3, with_parent=False, seed=77)
    b = irgl.irgl_batch_submit(tasks, cfg={"team": 8})
    irgl.irgl_batch_wait(b)
    for t, (gi, kind, s) in zip(tasks, meta):
        _, hg, _ = graphs[gi]
        alone, _, _ = irgl.query(hg, kind, s)
        assert torch.equal(alone, t.out), (gi, kind, s)


def test_batch_many_more_tasks_than_teams(irgl, graphs):
    g, hg, np_g = graphs[4]
    srcs = gg.pick_sources(g, 200, seed=5)
    tasks = [irgl.Task(hg, i % 2, s) for i, s in enumerate(srcs)]
    b = irgl.irgl_batch_submit(tasks, cfg={"team": 4, "grid": 16})
    stats = irgl.irgl_batch_wait(b)
    for t, st in zip(tasks, stats):
        assert st["status"] == 0
        np.testing.assert_array_equal(irgl.as_u32_numpy(t.out), _ref(t.kind, np_g, t.src))
