"""Autotuner for the batched launch and the open-batch server.

batch: picks the workgroup size (from T_control, the sizes both loop bodies
support), the team size and the grid-tier threshold by timing whole batches
of a workload built from a HELD-OUT seed, one coordinate at a time.
serve: picks the workgroup size, the team size, the gang threshold and the
gang queue depth by the p99 latency of a held-out Poisson query stream over
the resident graph set at 80% of the plain capacity.  The winner is cached per device and
workload class in a JSON file.

  python -m paper_1607_05707_amd.autotune --klass batch --seed 257
  python -m paper_1607_05707_amd.autotune --klass serve --seed 7
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

from . import graphgen as gg
from . import irgl

# tuned configurations, committed with the package (written by this module's main)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

DEFAULT = {"block": 256, "team": 16, "t_grid": 0}
SERVE_DEFAULT = {"block": 256, "team": 16, "gang_edges": 0, "gang_queue": 0}


def batch_tasks(seed: int, count: int, device, rmat_scale: int = 20, rmat_sources: int = 64,
                scale_cap=None):
    """The batched workload: `count` uniform random graphs (n log-uniform in
    [2^12, 2^20], mean degree in [4, 32], weights in [1, 1000]; BFS for even
    i, SSSP for odd i, one non-isolated source each) plus an R-MAT graph with
    `rmat_sources` BFS sources.  Returns (graphs kept alive, tasks)."""
    keep, tasks = [], []
    for g, kind, src in gg.config_batch(count, seed, device=device, scale_cap=scale_cap):
        hg = irgl.upload(g)
        keep.append((g, hg))
        tasks.append((hg, 0 if kind == "bfs" else 1, src))
    if rmat_sources:
        r = gg.rmat(rmat_scale, seed=seed * 10 + rmat_scale, weight_seed=seed * 10 + 1, wmax=255, device=device)
        hr = irgl.upload(r)
        keep.append((r, hr))
        for s in gg.pick_sources(r, rmat_sources, seed=seed * 10 + 2):
            tasks.append((hr, 0, s))
    return keep, tasks


def time_batch(tasks, cfg, reps: int = 2) -> float:
    """Best wall time (s) of the whole batch over `reps` runs."""
    objs = [irgl.Task(hg, k, s) for hg, k, s in tasks]
    ws = torch.empty(irgl.irgl_batch_workspace_bytes(objs, cfg), dtype=torch.uint8,
                     device=tasks[0][0].row_ptr.device)
    best = float("inf")
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = irgl.irgl_batch_submit(objs, ws=ws, cfg=cfg)
        stats = irgl.irgl_batch_wait(b)
        dt = time.perf_counter() - t0
        b.free()
        if any(s["status"] != 0 for s in stats):
            return float("inf")
        best = min(best, dt)
    return best


def tune(tasks, log=print):
    """Coordinate search from DEFAULT; returns (best config, its time)."""
    space = {
        "block": irgl.irgl_control_block_sizes(),
        "team": [4, 8, 16, 32, 64],
        "t_grid": [0, 512, 1024, 4096, 16384, -1],
    }
    cur = dict(DEFAULT)
    cur_t = time_batch(tasks, cur)
    log(f"[tune] start {cur} {cur_t * 1e3:.2f} ms")
    for key, values in space.items():
        for v in values:
            if v == cur[key]:
                continue
            cand = dict(cur)
            cand[key] = v
            try:
                t = time_batch(tasks, cand)
            except irgl.IrglError:
                continue
            log(f"[tune] {cand} {t * 1e3:.2f} ms")
            if t < cur_t:
                cur, cur_t = cand, t
    return cur, cur_t


def tune_serve(graphs, queries, arrivals, log=print, ring_cap: int = 512):
    """Coordinate search over the server configuration from SERVE_DEFAULT;
    objective: p99 latency, then p50.  Returns (best config, its summary)."""
    from . import serve
    space = {
        "block": [256, 512, 1024],
        "team": [8, 16, 32, 64],
        "gang_edges": [1 << 21, 1 << 22, 1 << 23, 1 << 24],
        "gang_queue": [0, 4, 16],
    }

    def score(cfg):
        lat, wall, _, rej = serve.run_served(graphs, queries, arrivals, 4 << 30, cfg=cfg, ring_cap=ring_cap)
        if rej:
            return (float("inf"), float("inf")), None
        summ = serve.summarize(lat, wall)
        return (summ["p99_ms"], summ["p50_ms"]), summ

    cur = dict(SERVE_DEFAULT)
    cur_s, cur_sum = score(cur)
    log(f"[tune serve] start {cur} {cur_sum}")
    for key, values in space.items():
        for v in values:
            if v == cur[key]:
                continue
            cand = dict(cur)
            cand[key] = v
            try:
                s, summ = score(cand)
            except irgl.IrglError:
                continue
            log(f"[tune serve] {cand} {summ}")
            if s < cur_s:
                cur, cur_s, cur_sum = cand, s, summ
    return cur, cur_sum


def cache_key(klass: str) -> str:
    name = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    return f"{name}/{klass}"


def load(klass: str):
    """The cached best config for this device and workload class, else the
    class default."""
    default = SERVE_DEFAULT if klass == "serve" else DEFAULT
    try:
        with open(CACHE) as f:
            return dict(json.load(f).get(cache_key(klass), default))
    except (OSError, ValueError):
        return dict(default)


def store(klass: str, cfg) -> None:
    data = {}
    try:
        with open(CACHE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        pass
    data[cache_key(klass)] = cfg
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=257,
                    help="held-out seed (the bench measures batch seed 256, serve stream seed 5)")
    ap.add_argument("--count", type=int, default=256, help="batch: tasks; serve: queries of the stream")
    ap.add_argument("--klass", default="batch", choices=["batch", "serve"])
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    if args.klass == "serve":
        from . import serve
        graphs = serve.resident_set("full", dev)
        capacity = serve.measure_capacity(graphs, serve.query_stream(graphs, 200, 6))
        queries = serve.query_stream(graphs, args.count, args.seed)
        arrivals = serve.poisson_arrivals(len(queries), 0.8 * capacity, args.seed + 1000)
        best, summ = tune_serve(graphs, queries, arrivals, log=lambda s: print(s, file=sys.stderr, flush=True))
        store("serve", best)
        print(json.dumps({"class": "serve", "config": best, "summary": summ,
                          "plain_capacity_qps": round(capacity, 1)}))
        return 0
    keep, tasks = batch_tasks(args.seed, args.count, dev)
    best, t = tune(tasks, log=lambda s: print(s, file=sys.stderr, flush=True))
    store(args.klass, best)
    print(json.dumps({"class": args.klass, "config": best, "ms": round(t * 1e3, 3)}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
