"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Levels and distances must match the oracle bit for bit; parents are not
unique and are checked by the validator's invariants.  Sizes span several
workgroup tiles with ragged tails, every nested-parallelism tier (by moving
the tier thresholds), both launch modes and all block sizes.
"""
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


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _check_query(irgl, g, hg, kind, src, cfg=None, with_parent=True, ref=None):
    rp, col, w = g.numpy()
    _say(f"{g.name} kind={kind} src={src} cfg={cfg}")
    out, par, st = irgl.query(hg, kind, src, with_parent=with_parent, cfg=cfg)
    got = irgl.as_u32_numpy(out)
    if ref is None:
        ref = oracle.bfs(rp, col, src)[0] if kind == BFS else oracle.dijkstra(rp, col, w, src)[0]
    np.testing.assert_array_equal(got, ref, err_msg=f"{g.name} kind={kind} src={src} cfg={cfg}")
    if with_parent:
        oracle.validate(rp, col, src, got, par.cpu().numpy(), None if kind == BFS else w)
    if kind == BFS:
        assert st["iterations"] == int(ref[ref != oracle.INF].max()) + 1
        assert st["frontier_edges"] == oracle.edges_scanned(rp, ref)
        assert st["items"] == int((ref != oracle.INF).sum())
        if not (cfg or {}).get("do_alpha") and not g.symmetric:
            assert st["edges"] == st["frontier_edges"]  # top-down scans every frontier edge
    assert st["status"] == 0
    return got, st


def _dev(g):
    return g.to(torch.device("cuda:0"))


def test_grid64_all_blocks_and_modes(irgl):
    g = _dev(gg.config_grid64())
    hg = irgl.upload(g)
    rp, col, w = g.numpy()
    ref_l = oracle.bfs(rp, col, 0)[0]
    ref_d = oracle.dijkstra(rp, col, w, 0)[0]
    golden = np.loadtxt(__file__.replace("test_gpu_parity.py", "golden/grid64_levels_hist.txt"),
                        dtype=np.int64)[:, 1]
    for block in (256, 512, 1024):
        for mode in (0, 1):
            cfg = {"block": block, "mode": mode}
            got, st = _check_query(irgl, g, hg, BFS, 0, cfg, ref=ref_l)
            np.testing.assert_array_equal(oracle.level_histogram(got), golden)
            assert st["iterations"] == 127
            _check_query(irgl, g, hg, SSSP, 0, cfg, ref=ref_d)


@pytest.mark.parametrize("t_wave,t_block,t_bitmap", [(64, 512, 0), (1, 1, 0), (1, 4, 1), (8, 64, 0),
                                                   (4096, 4096, 0), (64, 512, 0xFFFFFFFF)])
def test_rmat_tiers(irgl, t_wave, t_block, t_bitmap):
    g = _dev(gg.rmat(14, seed=3, weight_seed=4, wmax=255))
    hg = irgl.upload(g)
    cfg = {"t_wave": t_wave, "t_block": t_block, "t_bitmap": t_bitmap}
    for src in gg.pick_sources(g, 3, seed=5):
        _check_query(irgl, g, hg, BFS, src, cfg)
        _check_query(irgl, g, hg, SSSP, src, cfg)


@pytest.mark.parametrize("delta", [1, 7, 64, 0xFFFFFFFF])
def test_sssp_near_far_deltas(irgl, delta):
    g = _dev(gg.rmat(13, seed=21, weight_seed=22, wmax=255))
    hg = irgl.upload(g)
    for src in gg.pick_sources(g, 2, seed=23):
        for mode in (0, 1):
            _check_query(irgl, g, hg, SSSP, src, {"delta": delta, "mode": mode, "block": 256})
    r = _dev(gg.config_road(width=128))
    hr = irgl.upload(r)
    _check_query(irgl, r, hr, SSSP, r.sources[1], {"delta": delta})


@pytest.mark.parametrize("scale", [12, 15])
def test_bfs_direction_optimized(irgl, scale):
    """Bottom-up invocations (symmetric graphs) give the same levels, valid
    parents, and fewer scanned edges than the top-down-only run."""
    g = _dev(gg.rmat(scale, seed=40 + scale, weight_seed=1))
    hg = irgl.upload(g)
    for src in gg.pick_sources(g, 3, seed=scale):
        _, st_do = _check_query(irgl, g, hg, BFS, src, {"do_alpha": 14, "do_beta": 24})
        _, st_td = _check_query(irgl, g, hg, BFS, src, {"do_alpha": 0xFFFFFFFF})
        _check_query(irgl, g, hg, BFS, src, {"do_alpha": 1, "do_beta": 1, "block": 1024})
        assert st_td["edges"] == st_td["frontier_edges"]
        if scale >= 15:
            assert st_do["edges"] < st_td["edges"]
    # a directed graph never pulls (in-edges unknown): same as top-down
    d = _dev(gg.random_directed(3000, 30000, seed=1, weight_seed=2))
    hd = irgl.upload(d)
    _, st = _check_query(irgl, d, hd, BFS, 0, {"do_alpha": 1})
    assert st["edges"] == st["frontier_edges"]


def test_tiny_random_graphs(irgl):
    rng = np.random.default_rng(77)
    for i in range(40):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 5 * n + 1))
        g = _dev(gg.random_directed(n, m, seed=500 + i, weight_seed=600 + i, wmax=30))
        hg = irgl.upload(g)
        src = int(rng.integers(0, n))
        _check_query(irgl, g, hg, BFS, src, {"block": 256})
        _check_query(irgl, g, hg, SSSP, src, {"block": 256, "t_wave": 2, "t_block": 3})


def test_star_hub_and_long_path(irgl):
    n = 200_001
    src = [0] * (n - 1) + list(range(1, n))
    dst = list(range(1, n)) + [0] * (n - 1)
    wts = list(range(1, n)) * 2
    g = _dev(gg.from_edges(n, src, dst, wts, name="star"))
    hg = irgl.upload(g)
    _check_query(irgl, g, hg, BFS, 0)
    _check_query(irgl, g, hg, BFS, 17)
    _check_query(irgl, g, hg, SSSP, 5)
    k = 20_000
    w = np.random.default_rng(1).integers(1, 100, k - 1).tolist()
    gp = _dev(gg.from_edges(k, list(range(k - 1)) + list(range(1, k)),
                            list(range(1, k)) + list(range(k - 1)), w + w, name="path"))
    hp = irgl.upload(gp)
    _check_query(irgl, gp, hp, BFS, 0)
    _check_query(irgl, gp, hp, SSSP, k // 3)


def test_small_frontier_wave_per_item_and_grid_tier(irgl):
    """A worklist with no more items than wavefronts is dealt one item per
    wavefront, and one with fewer items than threads sends every range of a
    round or more to the grid tier; both give the oracle's result with
    ranges of every size, several block sizes and thresholds."""
    rng = np.random.default_rng(11)
    degs = [100, 300, 700, 1500, 2500, 5000]
    src, dst = [], []
    nxt = 61
    for i in range(1, 61):
        src.append(0)
        dst.append(i)
        d = degs[i % len(degs)]
        src += [i] * d
        dst += list(range(nxt, nxt + d))
        nxt += d
    n = nxt
    # cross edges among the leaves, so that the third level is not a tree
    a = rng.integers(61, n, 20000).tolist()
    b = rng.integers(61, n, 20000).tolist()
    src += a
    dst += b
    w = rng.integers(1, 50, len(src)).tolist()
    g = _dev(gg.from_edges(n, src, dst, w, name="two_level"))
    hg = irgl.upload(g)
    for cfg in (None, {"block": 512}, {"block": 256, "mode": 1}, {"t_grid": 4096}, {"t_grid": -1},
                {"t_wave": 32, "t_block": 128, "t_grid": 1024}, {"grid": 7}):
        _check_query(irgl, g, hg, BFS, 0, cfg)
        _check_query(irgl, g, hg, SSSP, 0, cfg)


@pytest.mark.parametrize("barrier", [0, 1])
def test_barrier_schemes(irgl, barrier):
    """Per-XCD and per-workgroup barrier coherence give identical results,
    over many barriers (near/far SSSP with a small step) and every block size."""
    g = _dev(gg.rmat(14, seed=31, weight_seed=32, wmax=255))
    hg = irgl.upload(g)
    for src in gg.pick_sources(g, 2, seed=33):
        for block in (256, 512, 1024):
            _check_query(irgl, g, hg, BFS, src, {"barrier": barrier, "block": block})
            _check_query(irgl, g, hg, SSSP, src, {"barrier": barrier, "block": block, "delta": 16})
    r = _dev(gg.config_road(width=128))
    hr = irgl.upload(r)
    _check_query(irgl, r, hr, SSSP, r.sources[1], {"barrier": barrier, "delta": 50})
    _check_query(irgl, r, hr, BFS, r.sources[2], {"barrier": barrier, "grid": 37})


def test_reordered_upload(irgl):
    """Degree-sorted relabelling: the same levels and distances under caller
    ids, valid parents, and SSSP parents identical to the plain upload's
    (smallest caller-id tight predecessor), in every launch form."""
    g = _dev(gg.rmat(14, seed=51, weight_seed=52, wmax=255))
    hr = irgl.upload(g, reorder=True)
    hp = irgl.upload(g)
    assert hr.reordered
    for src in gg.pick_sources(g, 3, seed=53):
        for cfg in (None, {"mode": 1}, {"delta": 16}, {"block": 512, "do_alpha": 1, "do_beta": 1},
                    {"t_bitmap": 0xFFFFFFFF, "t_grid": -1}):
            _check_query(irgl, g, hr, BFS, src, cfg)
            _check_query(irgl, g, hr, SSSP, src, cfg)
        _, p1, _ = irgl.query(hr, SSSP, src, with_parent=True)
        _, p2, _ = irgl.query(hp, SSSP, src, with_parent=True)
        assert torch.equal(p1, p2)
        # a batch on the relabelled handle traverses the caller's arrays
        t = irgl.Task(hr, SSSP, src)
        b = irgl.irgl_batch_submit([t], cfg={"team": 8})
        irgl.irgl_batch_wait(b)
        assert torch.equal(t.out, irgl.query(hp, SSSP, src)[0])
    d = _dev(gg.random_directed(3000, 30000, seed=61, weight_seed=62))
    hd = irgl.upload(d, reorder=True)
    for src in (0, 1, 2999):
        _check_query(irgl, d, hd, BFS, src)
        _check_query(irgl, d, hd, SSSP, src)
    one = _dev(gg.from_edges(1, [], [], [], name="single"))
    h1 = irgl.upload(one, reorder=True)
    _check_query(irgl, one, h1, BFS, 0)
    nb = irgl.irgl_reorder_bytes(g.n, g.m, True)
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_graph_upload_reordered(g.row_ptr, g.col, g.w, 0,
                                         store=torch.empty(nb - 1, dtype=torch.uint8, device=g.row_ptr.device))
    assert e.value.status == irgl.IRGL_ERR_WORKSPACE_TOO_SMALL


def test_sssp_light_heavy_split(irgl):
    """Relabelled weighted graphs carry an SSSP copy whose rows are split into
    light and heavy edges at the graph's step; irgl_graph_set_delta forces a
    split on graphs too small to get one by default.  Distances equal the
    oracle's at every step (from one that makes every edge heavy to one that
    makes every edge light), with every block size, with parents, and with
    the step removed again; a query at another step runs without the split."""
    graphs = [_dev(gg.rmat(14, seed=81, weight_seed=82, wmax=255)),
              _dev(gg.config_road(width=96)),
              _dev(gg.uniform_random(20000, 12.0, seed=83, weight_seed=84, wmax=1000)),
              _dev(gg.random_directed(5000, 40000, seed=85, weight_seed=86, wmax=64))]
    for g in graphs:
        hr = irgl.upload(g, reorder=True)
        wmax = int(np.asarray(g.numpy()[2], dtype=np.uint32).max())
        srcs = gg.pick_sources(g, 2, seed=87) if g.sources is None or len(g.sources) < 2 else g.sources[:2]
        for delta in (1, 7, max(2, wmax // 4), max(2, wmax // 2), wmax + 1, 3 * wmax):
            irgl.irgl_graph_set_delta(hr, delta)
            assert irgl.irgl_graph_default_delta(hr) == delta
            for src in srcs:
                _check_query(irgl, g, hr, SSSP, src, None, with_parent=False)
            _check_query(irgl, g, hr, SSSP, srcs[0], {"block": 256}, with_parent=True)
            _check_query(irgl, g, hr, SSSP, srcs[0], {"block": 1024, "t_grid": 64}, with_parent=False)
        # a query at a step other than the partition's runs unsplit
        _check_query(irgl, g, hr, SSSP, srcs[1], {"delta": 5}, with_parent=False)
        # the split also under the host-loop form falls back to the unsplit loop
        _check_query(irgl, g, hr, SSSP, srcs[1], {"mode": 1}, with_parent=False)
        irgl.irgl_graph_set_delta(hr, irgl.IRGL_DELTA_NONE)
        assert irgl.irgl_graph_default_delta(hr) == irgl.IRGL_DELTA_NONE
        _check_query(irgl, g, hr, SSSP, srcs[0], None, with_parent=False)
    with pytest.raises(irgl.IrglError):
        irgl.irgl_graph_set_delta(hr, 0)


def _star_with_hub(leaves):
    """Source 0 joined to `leaves` leaves by weight-1 edges, and a hub (the
    last vertex) joined to every leaf by weight-100 edges; symmetric."""
    h = leaves + 1
    a = [0] * leaves + [h] * leaves
    b = list(range(1, leaves + 1)) * 2
    w = [1] * leaves + [100] * leaves
    g = gg.from_edges(leaves + 2, a + b, b + a, w + w, name=f"star{leaves}_hub")
    g.symmetric = True
    return g


def test_sssp_pull_heavy_pass(irgl):
    """On a split symmetric graph, a bucket whose listed vertices carry many
    heavy edges relaxes them as a pull: each vertex beyond the bucket reads its
    own heavy range for the bucket's vertices (stats heavy_pulls counts these
    passes).  A vertex beyond the bucket whose heavy range is longer than one
    thread's pull limit (1024 edges) sends that pass back to the push form.
    Distances equal the oracle's either way, with parents, at every block
    size; on an R-MAT graph over several steps and sources pulls do happen."""
    pulls = {}
    for leaves in (1000, 2000):
        g = _dev(_star_with_hub(leaves))
        hr = irgl.upload(g, reorder=True)
        irgl.irgl_graph_set_delta(hr, 10)
        for cfg in (None, {"block": 256}, {"block": 1024}):
            _, st = _check_query(irgl, g, hr, SSSP, 0, cfg, with_parent=True)
            pulls.setdefault(leaves, set()).add(st["heavy_pulls"])
    # the hub's 1000 heavy edges are pulled; its 2000 are pushed (one pass fewer)
    assert len(pulls[1000]) == 1 and len(pulls[2000]) == 1
    assert min(pulls[1000]) >= 1 and min(pulls[1000]) == min(pulls[2000]) + 1
    g = _dev(gg.rmat(14, seed=91, weight_seed=92, wmax=255))
    assert g.symmetric
    hr = irgl.upload(g, reorder=True)
    srcs = gg.pick_sources(g, 3, seed=93)
    total = 0
    for delta in (16, 64, 128):
        irgl.irgl_graph_set_delta(hr, delta)
        for src in srcs:
            _, st = _check_query(irgl, g, hr, SSSP, src, None, with_parent=False)
            total += st["heavy_pulls"]
        _, st = _check_query(irgl, g, hr, SSSP, srcs[0], {"block": 1024}, with_parent=True)
        total += st["heavy_pulls"]
    assert total > 0
    # not symmetric: the same graph declared directed never pulls
    g.symmetric = False
    hd = irgl.upload(g, reorder=True)
    irgl.irgl_graph_set_delta(hd, 64)
    _, st = _check_query(irgl, g, hd, SSSP, srcs[0], None, with_parent=False)
    assert st["heavy_pulls"] == 0


@pytest.mark.parametrize("reduce", [0, 1])
def test_topology_driven_iterate(irgl, reduce):
    """IRGL_MODE_TOPOLOGY (a ForAll over every node whose invocation returns
    ReduceAndReturn Any(changed), or All(unchanged), re-invoked While Any /
    Until All): the oracle's levels and distances and valid parents on graphs
    with hubs, a long-diameter grid, directed edges and a relabelled upload,
    over block sizes and grid-tier settings.  BFS takes max level + 1
    invocations and scans every edge of every reached vertex exactly once;
    every invocation visits all n vertices."""
    path = gg.from_edges(300, list(range(299)) + list(range(1, 300)), list(range(1, 300)) + list(range(299)),
                         [1 + i % 7 for i in range(299)] * 2, name="path300")
    cases = [(gg.rmat(12, seed=71, weight_seed=72, wmax=255), False),
             (gg.config_road(width=64), False),
             (gg.random_directed(2000, 16000, seed=73, weight_seed=74), False),
             (gg.rmat(13, seed=75, weight_seed=76, wmax=255), True),
             (path, False)]
    for g0, reorder in cases:
        g = _dev(g0)
        hg = irgl.upload(g, reorder=reorder)
        rp, col, w = g.numpy()
        for src in gg.pick_sources(g, 2, seed=77):
            for cfg in ({}, {"block": 512, "t_grid": -1}, {"block": 1024, "t_grid": 1024}):
                c = dict(cfg, mode=irgl.IRGL_MODE_TOPOLOGY, reduce=reduce)
                for kind in (BFS, SSSP):
                    _say(f"topology {g.name} reorder={reorder} kind={kind} src={src} cfg={c}")
                    out, par, st = irgl.query(hg, kind, src, with_parent=True, cfg=c)
                    got = irgl.as_u32_numpy(out)
                    ref = oracle.bfs(rp, col, src)[0] if kind == BFS else oracle.dijkstra(rp, col, w, src)[0]
                    np.testing.assert_array_equal(got, ref, err_msg=f"{g.name} kind={kind} src={src} cfg={c}")
                    oracle.validate(rp, col, src, got, par.cpu().numpy(), None if kind == BFS else w)
                    assert st["status"] == 0
                    assert st["items"] == g.n * st["iterations"]
                    if kind == BFS:
                        assert st["iterations"] == int(ref[ref != oracle.INF].max()) + 1
                        assert st["edges"] == oracle.edges_scanned(rp, ref)
    bad = irgl.irgl_config()
    bad.mode = irgl.IRGL_MODE_TOPOLOGY
    bad.reduce = 2
    g = _dev(gg.config_grid64())
    hg = irgl.upload(g)
    with pytest.raises(irgl.IrglError) as e:
        irgl.query(hg, BFS, 0, cfg=bad)
    assert e.value.status == irgl.IRGL_ERR_CONFIG


def test_road_grid_small(irgl):
    g = _dev(gg.config_road(width=256))
    hg = irgl.upload(g)
    for src in g.sources[:3]:
        _check_query(irgl, g, hg, BFS, src)
        _check_query(irgl, g, hg, SSSP, src)


def test_isolated_source_and_single_vertex(irgl):
    g = _dev(gg.from_edges(5, [0, 1], [1, 0], [3, 3], name="tiny"))
    hg = irgl.upload(g)
    _check_query(irgl, g, hg, BFS, 3)
    _check_query(irgl, g, hg, SSSP, 4)
    g1 = _dev(gg.from_edges(1, [], [], [], name="single"))
    hg1 = irgl.upload(g1)
    _check_query(irgl, g1, hg1, BFS, 0)


def test_determinism_repeats(irgl):
    g = _dev(gg.rmat(13, seed=9, weight_seed=10))
    hg = irgl.upload(g)
    rp, col, w = g.numpy()
    src = gg.pick_sources(g, 1, seed=1)[0]
    ref = oracle.dijkstra(rp, col, w, src)[0]
    refp = None
    for rep in range(10):
        out, par, st = irgl.query(hg, SSSP, src, with_parent=True)
        np.testing.assert_array_equal(irgl.as_u32_numpy(out), ref)
        p = par.cpu().numpy()
        if refp is None:
            refp = p
            oracle.validate(rp, col, src, ref, p, w)
        np.testing.assert_array_equal(p, refp)  # SSSP parents are the smallest tight id


def test_error_paths(irgl):
    dev = torch.device("cuda:0")
    g = _dev(gg.rmat(12, seed=1, weight_seed=2))
    hg = irgl.upload(g)
    src = gg.pick_sources(g, 1, seed=3)[0]
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = irgl.workspace(hg, SSSP)
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_bfs(hg, g.n, out, None, ws)
    assert e.value.status == irgl.IRGL_ERR_INVALID_ARGUMENT
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_bfs(hg, src, out, None, ws[:1000])
    assert e.value.status == irgl.IRGL_ERR_WORKSPACE_TOO_SMALL
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_bfs(hg, src, out, None, ws, cfg={"block": 384})
    assert e.value.status == irgl.IRGL_ERR_CONFIG
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_bfs(hg, src, out, None, ws, cfg={"barrier": 2})
    assert e.value.status == irgl.IRGL_ERR_CONFIG
    gu = irgl.irgl_graph_upload(g.row_ptr, g.col, None)
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_sssp(gu, src, out, None, ws)
    assert e.value.status == irgl.IRGL_ERR_NO_WEIGHTS
    # worklist overflow is reported, not written out of bounds
    _say("overflow knob")
    _, _, st = irgl.query(hg, BFS, src, cfg={"wl_capacity": 8}, check=False)
    assert st["status"] == irgl.IRGL_ERR_OVERFLOW
    # iteration limit
    _, _, st = irgl.query(hg, BFS, src, cfg={"max_iter": 2}, check=False)
    assert st["status"] == irgl.IRGL_ERR_ITERATION_LIMIT
    _, _, st = irgl.query(hg, BFS, src, cfg={"max_iter": 2, "mode": 1}, check=False)
    assert st["status"] == irgl.IRGL_ERR_ITERATION_LIMIT
    # malformed CSR caught by on-device validation
    bad_col = g.col.clone()
    bad_col[5] = g.n + 3
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_graph_upload(g.row_ptr, bad_col, g.w, irgl.IRGL_VALIDATE)
    assert e.value.status == irgl.IRGL_ERR_INVALID_GRAPH
    # distance overflow
    big = torch.full_like(g.w, 0x7FFFFFFF)
    gb = irgl.irgl_graph_upload(g.row_ptr, g.col, big)
    _say("distance overflow")
    _, _, st = irgl.query(gb, SSSP, src, check=False)
    assert st["status"] == irgl.IRGL_ERR_OVERFLOW


def test_watchdog_and_abort_forced_from_host(irgl):
    g = _dev(gg.grid2d(64))
    hg = irgl.upload(g)
    _say("watchdog immediate")
    _, _, st = irgl.query(hg, BFS, 0, cfg={"watchdog_ms": irgl.IRGL_WATCHDOG_IMMEDIATE, "grid": 8},
                          check=False)
    assert st["status"] == irgl.IRGL_ERR_WATCHDOG
    flag = torch.ones(1, dtype=torch.int32, pin_memory=True)
    _say("abort flag")
    _, _, st = irgl.query(hg, BFS, 0, cfg={"abort_flag": flag.data_ptr()}, check=False)
    assert st["status"] == irgl.IRGL_ERR_ABORTED
    # a cleared flag does not disturb the query
    flag.zero_()
    _check_query(irgl, g, hg, BFS, 0, {"abort_flag": flag.data_ptr()})


def _directed(g):
    """The same arrays uploaded without the symmetric promise."""
    g.symmetric = False
    return g


def _expected_default_delta(g, validated=True, partitioned=False):
    """The default near/far step written out from the graph's shape: mean
    weight W, mean out-degree D, largest out-degree X (host arrays);
    `partitioned`: a relabelled weighted upload (light/heavy SSSP copy)."""
    rp, col, w = g.numpy()
    if not validated or w is None or g.m == 0:
        return 0xFFFFFFFF
    mean_w = float(np.asarray(w, dtype=np.uint32).astype(np.uint64).sum()) / g.m
    mean_deg = g.m / g.n
    x = int(np.diff(rp).max())
    if mean_deg < 8.0:
        d = 32.0 * mean_w / max(1.0, mean_deg)
    elif x <= 16.0 * mean_deg:
        d = 16.0 * mean_w / mean_deg
    elif partitioned and g.symmetric and g.m >= 1 << 22:
        d = mean_w / 8.0
    elif partitioned and g.m >= 1 << 25:
        d = mean_w / 4.0
    elif partitioned and g.m >= 1 << 24:
        d = mean_w / 2.0
    elif not partitioned and g.m >= 1 << 26:
        d = mean_w
    else:
        return 0xFFFFFFFF
    return int(min(4.0e9, max(1.0, d)))


def test_default_near_far_step(irgl):
    cases = [
        (gg.uniform_random(1 << 14, 16.0, seed=61, weight_seed=62, wmax=1000), "near-regular, D 16"),
        (gg.uniform_random(1 << 14, 32.0, seed=63, weight_seed=64, wmax=1000), "near-regular, D 32"),
        (gg.rmat(14, seed=65, weight_seed=66, wmax=255), "scale-free, below 2^24 edges"),
        (gg.rmat(20, seed=70, weight_seed=71, wmax=255), "scale-free, symmetric, 2^24 to 2^25 edges"),
        (_directed(gg.rmat(20, seed=70, weight_seed=71, wmax=255)), "scale-free, declared directed, 2^24 to 2^25"),
        (gg.config_road(width=64), "road-like, D < 8"),
        (gg.rmat(12, seed=67), "unweighted"),
    ]
    seen = set()
    for g, what in cases:
        g = _dev(g)
        for reorder in (False, True):
            want = _expected_default_delta(g, partitioned=reorder and g.w is not None)
            _say(f"default near/far step: {what} ({g.name}), relabelled={reorder} -> {want}")
            assert irgl.irgl_graph_default_delta(irgl.upload(g, reorder=reorder)) == want, (what, reorder)
            seen.add(want == 0xFFFFFFFF)
        if g.w is not None:
            src = g.sources[0] if g.sources else 0
            _check_query(irgl, g, irgl.upload(g), SSSP, src, with_parent=False)
    assert seen == {True, False}
    # without the validation pass the shape is unknown: plain Bellman-Ford order
    g = _dev(gg.uniform_random(1 << 12, 16.0, seed=68, weight_seed=69, wmax=1000))
    assert irgl.irgl_graph_default_delta(irgl.upload(g, flags=0)) == 0xFFFFFFFF


def test_trace_records_the_body_each_invocation_ran(irgl):
    # One outlined launch picks a loop body per invocation at run time
    # (dynamic piping).  BFS on a symmetric R-MAT graph: top-down invocations
    # record their expansion's busy ticks (word 8), bottom-up ones the edges
    # they scanned but no busy ticks.  SSSP with a near/far step: far-to-near
    # transfer invocations start from an empty worklist and record nothing
    # past their first two words.
    dev = torch.device("cuda:0")
    k_words = 12
    for g, kind, what in ((_dev(gg.rmat(16, seed=71, weight_seed=72, wmax=255)), BFS, "rmat16 BFS"),
                          (_dev(gg.config_road(width=128)), SSSP, "road128 SSSP")):
        hg = irgl.upload(g)
        src = gg.pick_sources(g, 1, seed=73)[0]
        tr = torch.zeros(k_words * 4096 + 1, dtype=torch.int64, device=dev)
        _say(f"trace: {what} src={src}")
        out, _, st = irgl.query(hg, kind, src, with_parent=False, cfg={"trace": tr, "trace_len": tr.numel()})
        rp, col, w = g.numpy()
        ref = oracle.bfs(rp, col, src)[0] if kind == BFS else oracle.dijkstra(rp, col, w, src)[0]
        np.testing.assert_array_equal(irgl.as_u32_numpy(out), ref)
        it = st["iterations"]
        assert 0 < it < 4096
        t = tr.cpu().numpy()
        starts, sizes, scanned = t[0:k_words * it:k_words], t[1:k_words * it:k_words], t[2:k_words * it:k_words]
        busy = t[8:k_words * it:k_words]
        assert (np.diff(starts) >= 0).all() and t[k_words * it] >= starts[-1] > 0
        assert sizes[0] == 1 and int(sizes.sum()) == st["items"]
        assert int(scanned.sum()) <= st["edges"]
        assert not t[k_words * it + 1:].any()  # nothing written past the end tick
        khz = irgl.irgl_wallclock_khz()  # converts the ticks to time
        assert khz > 0 and 0 < (t[k_words * it] - starts[0]) / khz < 10_000
        if kind == BFS:
            assert ((sizes > 0) & (busy == 0) & (scanned > 0)).any(), "no bottom-up invocation"
            assert (busy > 0).any(), "no top-down invocation"
        else:
            assert irgl.irgl_graph_default_delta(hg) != 0xFFFFFFFF
            transfer = sizes == 0
            assert transfer.any(), "no transfer invocation"
            assert not t[:k_words * it].reshape(it, k_words)[transfer][:, 2:].any()
            assert (busy > 0).any() and (scanned > 0).any()
    # a trace shorter than the run: words past trace_len stay untouched
    g = _dev(gg.config_road(width=64))
    hg = irgl.upload(g)
    tr = torch.full((64,), -1, dtype=torch.int64, device=dev)
    _, _, st = irgl.query(hg, BFS, 0, with_parent=False, cfg={"trace": tr, "trace_len": 2 * k_words})
    assert st["iterations"] > 2
    assert (tr.cpu().numpy()[2 * k_words:] == -1).all()
    assert isinstance(irgl.irgl_last_hip_error(), int)
