"""Full-size parity: the benchmark's own workloads, in the launch
configurations the benchmark times, against the CPU oracle.

* RMAT-22 (scale 22, edge factor 16, symmetrized: n = 4,194,304,
  m = 128,313,176), degree-sorted relabelling at upload, the library's
  default configuration, one launch per query into one reused workspace,
  no parent output.  Sources are compared with the oracle element by
  element (BFS levels and level histograms on all 64, SSSP distances on 3);
  every one of the 64 SSSP outputs is pinned by the distance certificate
  (``oracle.certify``), which holds for exactly one distance vector; one
  BFS with parents checks the parent tree.  One source in the topology-driven
  and host-loop launch forms, against the oracle.  The minimum spanning forest of
  the same graph (packed atomic section) is compared with Kruskal's: weight,
  every CSR entry's mark and every vertex's component.
* the road-like 4096 x 4096 grid (16.7M vertices, weights up to 10000),
  with and without its long edges (the latter ~8,190 BFS levels in one
  launch): BFS and SSSP from source 0 against the oracle, and from the
  workload's 8 random sources by the distance certificate.
* the batched workload (320 tasks: 256 uniform graphs of uneven size plus
  R-MAT-20 with 64 BFS sources) in one launch with the stored batch
  configuration; every fourth task is compared with the oracle and every
  task is pinned by the distance certificate.
* the served workload (eight resident graphs up to 16.7M vertices) through
  the open-batch server with the stored serve configuration; a burst of 200
  queries, every sixteenth compared with the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_05707_amd import graphgen as gg

pytestmark = pytest.mark.gpu

BFS, SSSP = 0, 1
# the benchmark's per-query configuration: every field zero = library default
BENCH_CFG = {"block": 0, "t_wave": 0, "t_block": 0, "t_grid": 0, "t_bitmap": 0, "grid": 0, "mode": 0}


@pytest.fixture(scope="module")
def irgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_05707_amd import irgl as mod
    return mod


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def rmat22(irgl):
    dev = torch.device("cuda:0")
    g = gg.config_rmat22(device=dev, nsources=64)
    hg = irgl.upload(g, reorder=True)
    rp, col, w = g.numpy()
    assert (g.n, g.m) == (4194304, 128313176)
    return g, hg, rp, col, w


def _run(irgl, hg, fn, kind, src, out, ws, stats, parent=None):
    fn(hg, src, out, parent, ws, None, stats, BENCH_CFG)
    st = irgl.read_stats(stats)
    assert st["status"] == 0, irgl.irgl_status_string(st["status"])
    return irgl.as_u32_numpy(out).copy(), st


def test_rmat22_bfs_full_size(irgl, rmat22):
    g, hg, rp, col, _ = rmat22
    dev = hg.row_ptr.device
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = irgl.workspace(hg, BFS, False, BENCH_CFG)
    stats = irgl.stats_tensor(dev)
    for i in range(64):
        src = g.sources[i]
        _say(f"rmat22 BFS source #{i} ({src}), bench configuration")
        got, st = _run(irgl, hg, irgl.irgl_bfs, BFS, src, out, ws, stats)
        ref, _ = oracle.bfs(rp, col, src, with_parent=False)
        np.testing.assert_array_equal(got, ref, err_msg=f"rmat22 BFS source {src}")
        reached = ref != oracle.INF
        assert st["items"] == int(reached.sum())
        assert st["frontier_edges"] == oracle.edges_scanned(rp, ref)
        assert st["iterations"] == int(ref[reached].max()) + 1
        assert st["block"] == 1024
        np.testing.assert_array_equal(oracle.level_histogram(got), oracle.level_histogram(ref))
    # parents: any valid BFS tree; the validator checks it against the levels
    src = g.sources[1]
    _say(f"rmat22 BFS source #1 ({src}) with parents")
    wsp = irgl.workspace(hg, BFS, True, BENCH_CFG)
    par = torch.empty(g.n, dtype=torch.int32, device=dev)
    got, _ = _run(irgl, hg, irgl.irgl_bfs, BFS, src, out, wsp, stats, parent=par)
    oracle.validate(rp, col, src, got, par.cpu().numpy())


def test_rmat22_sssp_full_size(irgl, rmat22):
    g, hg, rp, col, w = rmat22
    dev = hg.row_ptr.device
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = irgl.workspace(hg, SSSP, False, BENCH_CFG)
    stats = irgl.stats_tensor(dev)
    # symmetric scale-free with more than 2^22 edges, relabelled weighted
    # upload (rows split into light and heavy edges): the near/far step is an
    # eighth of the mean weight
    mean_w = float(np.asarray(w, dtype=np.uint32).astype(np.uint64).sum()) / g.m
    assert irgl.irgl_graph_default_delta(hg) == int(mean_w / 8.0)
    compare = (0, 31, 63)
    for i in range(64):
        src = g.sources[i]
        _say(f"rmat22 SSSP source #{i} ({src}), bench configuration")
        got, st = _run(irgl, hg, irgl.irgl_sssp, SSSP, src, out, ws, stats)
        assert st["block"] == 512
        oracle.certify(rp, col, src, got, w)
        if i in compare:
            ref, _ = oracle.dijkstra(rp, col, w, src, with_parent=False)
            np.testing.assert_array_equal(got, ref, err_msg=f"rmat22 SSSP source {src}")


def test_rmat22_topology_driven_and_host_loop_full_size(irgl, rmat22):
    # the other two launch forms on the same graph and source: topology-driven
    # Iterate (every invocation a ForAll over all vertices, ReduceAndReturn Any)
    # and one launch per invocation from the host
    g, hg, rp, col, w = rmat22
    dev = hg.row_ptr.device
    src = g.sources[5]
    refs = {BFS: oracle.bfs(rp, col, src, with_parent=False)[0],
            SSSP: oracle.dijkstra(rp, col, w, src, with_parent=False)[0]}
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    stats = irgl.stats_tensor(dev)
    for mode in (irgl.IRGL_MODE_TOPOLOGY, irgl.IRGL_MODE_HOST_LOOP):
        for kind, fn in ((BFS, irgl.irgl_bfs), (SSSP, irgl.irgl_sssp)):
            cfg = {"mode": mode}
            _say(f"rmat22 kind={kind} source #5 ({src}) mode={mode}")
            ws = irgl.workspace(hg, kind, False, cfg)
            fn(hg, src, out, None, ws, None, stats, cfg)
            st = irgl.read_stats(stats)
            assert st["status"] == 0, irgl.irgl_status_string(st["status"])
            np.testing.assert_array_equal(irgl.as_u32_numpy(out), refs[kind],
                                          err_msg=f"rmat22 kind={kind} mode={mode}")
            if mode == irgl.IRGL_MODE_TOPOLOGY:
                assert st["items"] == g.n * st["iterations"]


def test_rmat22_spanning_forest_full_size(irgl, rmat22):
    # the benchmark's forest: the relabelled handle, packed atomic section,
    # default configuration; results refer to the caller's ids and entries
    g, hg, rp, col, w = rmat22
    _say("rmat22 minimum spanning forest, packed atomic section")
    weight, comp, in_forest, st = irgl.mst(hg, cfg={"lock": irgl.IRGL_LOCK_PACKED})
    assert st["status"] == 0
    ref_w, ref_f, ref_c, ref_ne = oracle.kruskal(rp, col, w)
    assert weight == ref_w
    assert st["frontier_edges"] == ref_ne
    np.testing.assert_array_equal(comp.cpu().numpy(), ref_c)
    np.testing.assert_array_equal(in_forest.cpu().numpy(), ref_f)


@pytest.mark.parametrize("long_edges", [True, False])
def test_road4096_full_size(irgl, long_edges):
    # the road-like 4096 x 4096 grid (16.7M vertices), relabelled upload and
    # default configuration; without the long edges BFS runs ~8,190 levels,
    # one grid barrier each, in one launch
    dev = torch.device("cuda:0")
    g = gg.config_road(device=dev, long_edges=long_edges)
    hg = irgl.upload(g, reorder=True)
    rp, col, w = g.numpy()
    assert len(g.sources) == 9
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    stats = irgl.stats_tensor(dev)
    for kind, fn in ((BFS, irgl.irgl_bfs), (SSSP, irgl.irgl_sssp)):
        ws = irgl.workspace(hg, kind, False, BENCH_CFG)
        for i, src in enumerate(g.sources):
            _say(f"{g.name} kind={kind} source #{i} ({src}), default configuration")
            got, st = _run(irgl, hg, fn, kind, src, out, ws, stats)
            oracle.certify(rp, col, src, got, w if kind == SSSP else None)
            if i == 0:
                ref = oracle.bfs(rp, col, src, with_parent=False)[0] if kind == BFS else \
                    oracle.dijkstra(rp, col, w, src, with_parent=False)[0]
                np.testing.assert_array_equal(got, ref, err_msg=f"{g.name} kind={kind}")
            if kind == BFS:
                assert st["iterations"] == int(got[got != oracle.INF].max()) + 1
                if not long_edges and i == 0:
                    # from the corner the high-diameter grid has ~8,190 levels
                    assert st["iterations"] > 8000


def test_batched_workload_full_size(irgl):
    from paper_1607_05707_amd import autotune
    dev = torch.device("cuda:0")
    keep, tasks = autotune.batch_tasks(256, 256, dev)
    assert len(tasks) == 320
    cfg = autotune.load("batch")
    objs = [irgl.Task(hg, k, s) for hg, k, s in tasks]
    _say(f"batched workload, {len(objs)} tasks, configuration {cfg}")
    b = irgl.irgl_batch_submit(objs, cfg=cfg)
    stats = irgl.irgl_batch_wait(b)
    b.free()
    assert all(s["status"] == 0 for s in stats)
    host = {}
    for i, t in enumerate(objs):
        gi = next(j for j, (_, hg) in enumerate(keep) if hg is t.g)
        if gi not in host:
            host[gi] = keep[gi][0].numpy()
        rp, col, w = host[gi]
        got = irgl.as_u32_numpy(t.out)
        oracle.certify(rp, col, t.src, got, w if t.kind == SSSP else None)
        if t.kind == BFS:
            assert stats[i]["frontier_edges"] == oracle.edges_scanned(rp, got)
        if i % 4 == 0:
            ref = oracle.bfs(rp, col, t.src, with_parent=False)[0] if t.kind == BFS else \
                oracle.dijkstra(rp, col, w, t.src, with_parent=False)[0]
            np.testing.assert_array_equal(got, ref, err_msg=f"batched task {i} kind={t.kind} src={t.src}")


def test_served_workload_full_size(irgl):
    from paper_1607_05707_amd import autotune, serve
    dev = torch.device("cuda:0")
    graphs = serve.resident_set("full", dev)
    queries = serve.query_stream(graphs, 200, 5)
    keep = set(range(0, len(queries), 16))
    cfg = autotune.load("serve")
    _say(f"served workload, {len(queries)} queries in one burst, configuration {cfg}")
    lat, _, kept, rejected = serve.run_served(graphs, queries, np.zeros(len(queries)), 4 << 30, cfg=cfg,
                                              keep_outputs=keep)
    assert rejected == 0 and not np.isnan(lat).any()
    assert set(kept) == keep
    host = {}
    for qi in sorted(keep):
        gi, kind, src = queries[qi]
        if gi not in host:
            host[gi] = graphs[gi][0].numpy()
        rp, col, w = host[gi]
        _say(f"served query {qi}: {graphs[gi][0].name} kind={kind} src={src}")
        ref = oracle.bfs(rp, col, src, with_parent=False)[0] if kind == BFS else \
            oracle.dijkstra(rp, col, w, src, with_parent=False)[0]
        np.testing.assert_array_equal(irgl.as_u32_numpy(kept[qi]), ref, err_msg=f"served query {qi}")


def test_dmr_full_size(irgl):
    # the benchmark's mesh refinement: 1M random points in the unit square
    # (2M triangles), default configuration (30 degrees, 256-thread
    # workgroups, co-resident grid); the whole refined mesh is checked
    from oracle import mesh as om
    from paper_1607_05707_amd import meshgen
    m = meshgen.random_square(1_000_000, 42)
    _say(f"dmr {m.name}: {m.npts} points, {m.ntri} triangles, default configuration")
    dm = irgl.DeviceMesh.from_host(m, torch.device("cuda:0"))
    st = irgl.dmr(dm)
    assert st["final_bad"] == 0 and st["block"] == 256
    res = om.check_mesh(dm.pts[:dm.npts].cpu().numpy(), dm.tri[:dm.ntri].cpu().numpy(),
                        dm.nbr[:dm.ntri].cpu().numpy(), input_pts=m.input_pts, min_angle=30.0)
    assert res["triangles"] == dm.ntri > 4 * m.ntri
