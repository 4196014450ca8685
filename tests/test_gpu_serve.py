"""Open batches (serving): tasks enqueued while the server kernel runs must
give the same result as alone and as the oracle; ring-full and idle-exit /
relaunch paths; the serving loop with memory admission."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1607_05707_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def irgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_05707_amd import irgl as mod
    return mod


@pytest.fixture(scope="module")
def graphs(irgl):
    dev = torch.device("cuda:0")
    gs = [gg.rmat(12, seed=31, weight_seed=32), gg.config_road(width=80), gg.config_grid64(),
          gg.uniform_random(3000, 8.0, seed=33, weight_seed=34, wmax=500)]
    return [(g.to(dev), irgl.upload(g.to(dev)), g.numpy()) for g in gs]


def _ref(kind, np_g, src):
    rp, col, w = np_g
    return oracle.bfs(rp, col, src)[0] if kind == 0 else oracle.dijkstra(rp, col, w, src)[0]


def _wait(irgl, server, tickets, timeout=30.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                st = irgl.irgl_batch_poll(server, t)
                if st is not None:
                    out[t] = st
        assert time.time() - t0 < timeout, (f"server did not finish: {sorted(set(tickets) - set(out))} pending, "
                                            f"(launches, gave up at start) = {irgl.irgl_batch_launches(server)}")
    return out


def test_server_results_match_oracle_and_alone(irgl, graphs):
    server = irgl.irgl_batch_open([hg for _, hg, _ in graphs], cfg={"team": 8}, ring_cap=64)
    rng = np.random.default_rng(1)
    tasks, tickets = [], []
    for i in range(60):
        gi = int(rng.integers(0, len(graphs)))
        g, hg, np_g = graphs[gi]
        src = gg.pick_sources(g, 50, seed=gi)[int(rng.integers(0, 50))]
        t = irgl.Task(hg, int(rng.integers(0, 2)), src, with_parent=(i % 3 == 0))
        tk = irgl.irgl_batch_enqueue(server, t)
        assert tk is not None
        tasks.append((gi, t))
        tickets.append(tk)
    stats = _wait(irgl, server, tickets)
    for (gi, t), tk in zip(tasks, tickets):
        g, hg, np_g = graphs[gi]
        assert stats[tk]["status"] == 0
        got = irgl.as_u32_numpy(t.out)
        np.testing.assert_array_equal(got, _ref(t.kind, np_g, t.src))
        alone, _, _ = irgl.query(hg, t.kind, t.src)
        assert torch.equal(alone, t.out)
        if t.parent is not None:
            rp, col, w = np_g
            oracle.validate(rp, col, t.src, got, t.parent.cpu().numpy(), None if t.kind == 0 else w)
    server.close()


@pytest.mark.parametrize("gang_edges,team,gang_queue,barrier", [(20_000, 8, 0, 0), (1, 4, 0, 0),
                                                                (20_000, 10_000, 0, 0), (1 << 30, 8, 6, 0),
                                                                (20_000, 8, 0, 1), (1, 4, 0, 1)])
def test_gang_tasks_in_the_mix(irgl, graphs, gang_edges, team, gang_queue, barrier):
    """Tasks on graphs with at least gang_edges edges (or enqueued while fewer
    than gang_queue are in flight) run on the whole grid between the teams'
    own tasks; every result equals the oracle, in ring order or not, and the
    kernel ends and relaunches between waves."""
    print(f"[case] gang_edges={gang_edges} team={team} gang_queue={gang_queue} barrier={barrier}", flush=True)
    server = irgl.irgl_batch_open([hg for _, hg, _ in graphs],
                                  cfg={"team": team, "gang_edges": gang_edges, "gang_queue": gang_queue,
                                       "barrier": barrier},
                                  ring_cap=32, idle_ms=5)
    rng = np.random.default_rng(gang_edges + team)
    for wave in range(2):
        tasks, tickets, stats = [], [], {}
        t0 = time.time()
        for i in range(40):
            gi = int(rng.integers(0, len(graphs)))
            g, hg, np_g = graphs[gi]
            src = gg.pick_sources(g, 50, seed=gi)[int(rng.integers(0, 50))]
            t = irgl.Task(hg, int(rng.integers(0, 2)), src, with_parent=(i % 4 == 0))
            while True:
                tk = irgl.irgl_batch_enqueue(server, t)
                if tk is not None:
                    break
                for old in tickets:  # make room: a slot is reused once its task was polled done
                    if old not in stats:
                        st = irgl.irgl_batch_poll(server, old)
                        if st is not None:
                            stats[old] = st
                assert time.time() - t0 < 30.0, (sorted(set(tickets) - set(stats)),
                                                  irgl.irgl_batch_launches(server))
            tasks.append((gi, t))
            tickets.append(tk)
        stats.update(_wait(irgl, server, [tk for tk in tickets if tk not in stats]))
        for (gi, t), tk in zip(tasks, tickets):
            g, hg, np_g = graphs[gi]
            st = stats[tk]
            assert st["status"] == 0
            ref = _ref(t.kind, np_g, t.src)
            got = irgl.as_u32_numpy(t.out)
            np.testing.assert_array_equal(got, ref, err_msg=f"graph {gi} kind {t.kind} src {t.src}")
            if t.kind == 0:
                assert st["frontier_edges"] == oracle.edges_scanned(np_g[0], ref)
            if t.parent is not None:
                rp, col, w = np_g
                oracle.validate(rp, col, t.src, got, t.parent.cpu().numpy(), None if t.kind == 0 else w)
        print(f"[wave {wave}] (launches, gave up at start) = {irgl.irgl_batch_launches(server)}", flush=True)
        time.sleep(0.05)  # idle: the kernel ends, the next wave relaunches it
    server.close()


def test_ring_full_then_drain_and_idle_relaunch(irgl, graphs):
    g, hg, np_g = graphs[0]
    server = irgl.irgl_batch_open([hg], cfg={"team": 4}, ring_cap=4, idle_ms=5)
    srcs = gg.pick_sources(g, 20, seed=3)
    tasks = []
    pending = set()
    busy_seen = False
    t0 = time.time()
    for s in srcs:
        t = irgl.Task(hg, 1, s)
        while True:
            tk = irgl.irgl_batch_enqueue(server, t)
            if tk is not None:
                break
            busy_seen = True
            for old in list(pending):  # make room: finished slots can be reused
                if irgl.irgl_batch_poll(server, old) is not None:
                    pending.discard(old)
            assert time.time() - t0 < 30.0
        pending.add(tk)
        tasks.append(t)
    _wait(irgl, server, sorted(pending))
    time.sleep(0.1)  # the server kernel ends after idle_ms without work
    t = irgl.Task(hg, 0, srcs[0])
    tk = irgl.irgl_batch_enqueue(server, t)
    _wait(irgl, server, [tk])
    for t in tasks + [t]:
        np.testing.assert_array_equal(irgl.as_u32_numpy(t.out), _ref(t.kind, np_g, t.src))
    assert busy_seen
    server.close()


def test_serving_loop_alone_equals_in_the_mix(irgl):
    from paper_1607_05707_amd import serve
    dev = torch.device("cuda:0")
    graphs = serve.resident_set("small", dev)
    queries = serve.query_stream(graphs, 300, seed=9)
    arrivals = serve.poisson_arrivals(len(queries), 3000.0, seed=10)
    keep = set(range(0, 300, 7))
    lat, wall, kept, rej = serve.run_served(graphs, queries, arrivals, budget_bytes=1 << 20, cfg={"team": 8},
                                            keep_outputs=keep)
    assert rej == 0 and not np.isnan(lat).any()
    for qi in sorted(keep):
        gi, kind, src = queries[qi]
        alone, _, _ = irgl.query(graphs[gi][1], kind, src)
        assert torch.equal(alone, kept[qi]), qi
