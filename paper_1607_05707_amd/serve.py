"""Serving loop: continuous batching of BFS/SSSP queries over device-resident graphs.

A seeded Poisson stream of queries (graph uniform over the resident set, kind
50/50, source uniform over non-isolated vertices) arrives at a fixed rate.
The serving loop admits a query when its output buffers fit the
device-memory budget for per-query state (otherwise it waits; a query that
can never fit is rejected), enqueues it on an open batch (irgl_batch_open:
a persistent kernel whose teams take tasks while others are running) and
polls for completions.  Latency is arrival -> completion on the host's
monotonic clock, so it includes queueing.

The comparator ("plain") serves the same arrival stream FIFO with one
irgl_bfs / irgl_sssp launch per query on one stream.

  python -m paper_1607_05707_amd.serve [--set full|small] [--queries N]
                                       [--lambdas 0.25,0.5,0.8,0.95] [--budget-gb 4]
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from collections import deque

import numpy as np
import torch

from . import graphgen as gg
from . import irgl


def resident_set(kind: str, device):
    """The served graphs.  full: RMAT scales 16/18/20/22, road-like grids
    1024^2/2048^2/4096^2, uniform n=2^20 degree 16.  small: a quick stand-in."""
    if kind == "full":
        specs = [("rmat16", lambda: gg.rmat(16, seed=16, weight_seed=1601, wmax=255, device=device)),
                 ("rmat18", lambda: gg.rmat(18, seed=18, weight_seed=1801, wmax=255, device=device)),
                 ("rmat20", lambda: gg.rmat(20, seed=20, weight_seed=2001, wmax=255, device=device)),
                 ("rmat22", lambda: gg.rmat(22, seed=22, weight_seed=2201, wmax=255, device=device)),
                 ("road1024", lambda: gg.config_road(width=1024, device=device)),
                 ("road2048", lambda: gg.config_road(width=2048, device=device)),
                 ("road4096", lambda: gg.config_road(width=4096, device=device)),
                 ("uniform20", lambda: gg.uniform_random(1 << 20, 16.0, seed=5, weight_seed=6, wmax=255,
                                                         device=device))]
    else:
        specs = [("rmat12", lambda: gg.rmat(12, seed=12, weight_seed=1201, wmax=255, device=device)),
                 ("rmat14", lambda: gg.rmat(14, seed=14, weight_seed=1401, wmax=255, device=device)),
                 ("road128", lambda: gg.config_road(width=128, device=device)),
                 ("uniform14", lambda: gg.uniform_random(1 << 14, 16.0, seed=5, weight_seed=6, wmax=255,
                                                         device=device))]
    out = []
    for name, make in specs:
        g = make()
        g.name = name
        out.append((g, irgl.upload(g)))
    return out


def query_stream(graphs, count: int, seed: int):
    """[(graph index, kind, source)] drawn with a seeded generator."""
    rng = np.random.default_rng(seed)
    pools = [gg.pick_sources(g, 4096, seed=seed + i) for i, (g, _) in enumerate(graphs)]
    qs = []
    for _ in range(count):
        gi = int(rng.integers(0, len(graphs)))
        kind = int(rng.integers(0, 2))
        src = pools[gi][int(rng.integers(0, len(pools[gi])))]
        qs.append((gi, kind, src))
    return qs


def state_bytes(g) -> int:
    """Per-query device state: the output array the caller allocates for the
    query.  Everything else a running query touches (worklists, stamps, far
    lists, bitmap) lives in the server's team scratch, allocated once when the
    server opens and reused by every query, so it is not per-query state."""
    return 4 * g.n


def run_plain(graphs, queries, arrivals):
    """FIFO, one launch per query, same arrival stream.  Returns latencies (s)."""
    dev = graphs[0][0].row_ptr.device
    ws = {}
    outs = {}
    for gi, (g, hg) in enumerate(graphs):
        for k in (0, 1):
            ws[(gi, k)] = irgl.workspace(hg, k)
        outs[gi] = torch.empty(g.n, dtype=torch.int32, device=dev)
    lat = []
    t0 = time.perf_counter()
    for (gi, kind, src), a in zip(queries, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        fn = irgl.irgl_bfs if kind == 0 else irgl.irgl_sssp
        fn(graphs[gi][1], src, outs[gi], None, ws[(gi, kind)])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - a)
    return np.array(lat), time.perf_counter() - t0


def run_served(graphs, queries, arrivals, budget_bytes: int, cfg=None, ring_cap: int = 512,
               keep_outputs=None, info=None):
    """Continuous batching through an open batch.  Returns latencies (s), wall
    time, the outputs of the queries whose indices are in keep_outputs, and
    the number rejected.  `info` (a dict), when given, receives the admission
    record: queries that waited for memory, the peak of admitted state bytes
    and of queries in flight."""
    hgs = [hg for _, hg in graphs]
    server = irgl.irgl_batch_open(hgs, cfg=cfg, ring_cap=ring_cap)
    dev = graphs[0][0].row_ptr.device
    pending = deque()          # arrived, not yet admitted
    inflight = {}              # ticket -> (query index, task, bytes)
    lat = np.zeros(len(queries))
    used = 0
    kept = {}
    nxt = 0
    done_count = 0
    rejected = 0
    mem_waited = set()
    peak_used = 0
    peak_inflight = 0
    t0 = time.perf_counter()
    while done_count + rejected < len(queries):
        now = time.perf_counter() - t0
        while nxt < len(queries) and arrivals[nxt] <= now:
            pending.append(nxt)
            nxt += 1
        # admission by memory budget (FIFO: the head waits if it does not fit)
        while pending:
            qi = pending[0]
            gi, kind, src = queries[qi]
            need = state_bytes(graphs[gi][0])
            if need > budget_bytes:
                pending.popleft()
                rejected += 1
                lat[qi] = np.nan
                continue
            if used + need > budget_bytes:
                mem_waited.add(qi)
                break
            task = irgl.Task(hgs[gi], kind, src)
            ticket = irgl.irgl_batch_enqueue(server, task)
            if ticket is None:  # ring full
                break
            pending.popleft()
            used += need
            inflight[ticket] = (qi, task, need)
            peak_used = max(peak_used, used)
            peak_inflight = max(peak_inflight, len(inflight))
        for ticket in list(inflight):
            st = irgl.irgl_batch_poll(server, ticket)
            if st is not None:
                qi, task, need = inflight.pop(ticket)
                lat[qi] = time.perf_counter() - t0 - arrivals[qi]
                if st["status"] != 0:
                    raise RuntimeError(f"query {qi} failed: {irgl.irgl_status_string(st['status'])}")
                if keep_outputs is not None and qi in keep_outputs:
                    kept[qi] = task.out.clone()
                    # the buffer is recycled by the allocator once the task is dropped
                    torch.cuda.current_stream(dev).synchronize()
                used -= need
                done_count += 1
        if not inflight and not pending and nxt < len(queries):
            gap = arrivals[nxt] - (time.perf_counter() - t0)
            if gap > 0.0005:
                time.sleep(gap - 0.0002)
    wall = time.perf_counter() - t0
    server.close()
    torch.cuda.synchronize()
    if info is not None:
        info.update({"waited_for_memory": len(mem_waited), "peak_state_bytes": peak_used,
                     "peak_in_flight": peak_inflight})
    return lat, wall, kept, rejected


def poisson_arrivals(count: int, rate: float, seed: int):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def summarize(lat, wall):
    good = lat[~np.isnan(lat)]
    return {"p50_ms": round(float(np.percentile(good, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(good, 99)) * 1e3, 3),
            "qps": round(len(good) / wall, 1)}


def measure_capacity(graphs, queries):
    """Plain service rate: back-to-back single launches (queries per second)."""
    lat, wall = run_plain(graphs, queries, np.zeros(len(queries)))
    return len(queries) / wall


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", default="full", choices=["full", "small"])
    ap.add_argument("--queries", type=int, default=2000)
    ap.add_argument("--lambdas", default="0.25,0.5,0.8,0.95")
    ap.add_argument("--budget-gb", type=float, default=4.0)
    ap.add_argument("--team", type=int, default=16)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    graphs = resident_set(args.set, dev)
    print(f"[serve] {len(graphs)} graphs resident: "
          + ", ".join(f"{g.name}(n={g.n}, m={g.m})" for g, _ in graphs), file=sys.stderr, flush=True)
    cap_q = query_stream(graphs, min(200, args.queries), args.seed + 1)
    capacity = measure_capacity(graphs, cap_q)
    print(f"[serve] plain capacity {capacity:.1f} queries/s", file=sys.stderr, flush=True)
    results = {"capacity_qps": round(capacity, 1), "lambdas": {}}
    queries = query_stream(graphs, args.queries, args.seed)
    for frac in [float(x) for x in args.lambdas.split(",")]:
        arr = poisson_arrivals(args.queries, frac * capacity, args.seed + 7)
        lat_s, wall_s, _, rej = run_served(graphs, queries, arr, int(args.budget_gb * 2 ** 30),
                                           cfg={"team": args.team})
        lat_p, wall_p = run_plain(graphs, queries, arr)
        results["lambdas"][str(frac)] = {"served": summarize(lat_s, wall_s), "plain": summarize(lat_p, wall_p),
                                        "rejected": rej}
        print(f"[serve] lambda={frac}: served {results['lambdas'][str(frac)]['served']} "
              f"plain {results['lambdas'][str(frac)]['plain']}", file=sys.stderr, flush=True)
    print(json.dumps(results), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
