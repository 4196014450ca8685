"""Throughput bench of the data-driven BFS/SSSP hot path on one MI355X.

A step is one pass of the whole path over one batch of queries: for every
source of the workload, one BFS and one SSSP (init + outlined persistent
Iterate loop + nested edge scheduler + cooperative pushes), each its own
`irgl_bfs` / `irgl_sssp` call on one stream ("plain" form).

Metric: GTEPS = sum over queries of m_cc / time, where m_cc is the number of
directed CSR entries an exact top-down traversal from the source scans
(sum of out-degrees of the reached vertices; SSSP uses the same numerator).

Prints ONE JSON line.  Inputs are synthetic (seeded R-MAT, grid, road-like
grid) and already resident in HBM when the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(kind: int, n: int, reached: int, m_cc: int) -> int:
    """Algorithmic HBM bytes of one query: what the method itself must move.

    BFS:  4n (level init) + 20 B per reached vertex (pop 4, row offsets 8,
          level write 4, push 4) + 8 B per scanned edge (col 4, probe 4).
    SSSP: 4n + 28 B per reached vertex (pop 4, row offsets 8, dist read 4,
          atomicMin 4, stamp 4, push 4) + 12 B per edge (col 4, weight 4,
          probe 4), counted once per edge of the reached component."""
    if kind == 0:
        return 4 * n + 20 * reached + 8 * m_cc
    return 4 * n + 28 * reached + 12 * m_cc


def host_cpu():
    """CPU model and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(g, sources, budget_s: float, gpu_results, reps: int = 5):
    """Time the CPU oracle (one thread) on a bounded sample of the workload:
    the median of `reps` runs per source and kind, source after source until
    the budget is spent."""
    import statistics

    import numpy as np
    import oracle
    rp, col, w = g.numpy()
    t_bfs = t_sssp = 0.0
    e_bfs = e_sssp = 0
    nb = ns = 0
    parity = True
    t_start = time.perf_counter()
    for src in sources:
        runs = []
        for _ in range(reps):
            t0 = time.perf_counter()
            lv, _ = oracle.bfs(rp, col, src, with_parent=False)
            runs.append(time.perf_counter() - t0)
        t_bfs += statistics.median(runs)
        mcc = oracle.edges_scanned(rp, lv)
        e_bfs += mcc
        nb += 1
        if src in gpu_results:
            parity &= bool(np.array_equal(gpu_results[src][0], lv))
        if w is not None:
            runs = []
            for _ in range(reps):
                t0 = time.perf_counter()
                d, _ = oracle.dijkstra(rp, col, w, src, with_parent=False)
                runs.append(time.perf_counter() - t0)
            t_sssp += statistics.median(runs)
            e_sssp += mcc
            ns += 1
            if src in gpu_results:
                parity &= bool(np.array_equal(gpu_results[src][1], d))
        if time.perf_counter() - t_start > budget_s:
            break
    total_t = t_bfs + t_sssp
    model, nproc, usable = host_cpu()
    return {
        "value": round((e_bfs + e_sssp) / total_t / 1e9, 4) if total_t > 0 else None,
        "unit": "GTEPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nb} BFS + {ns} SSSP queries (serial queue BFS, binary-heap Dijkstra) "
                  f"from the first {nb} sources of the same graph, median of {reps} runs each, "
                  f"one host thread, {time.perf_counter() - t_start:.1f} s wall",
        "cpu_model": model,
        "nproc": nproc,
        "usable_threads": usable,
        "bfs_gteps": round(e_bfs / t_bfs / 1e9, 4) if t_bfs > 0 else None,
        "sssp_gteps": round(e_sssp / t_sssp / 1e9, 4) if t_sssp > 0 else None,
    }, parity


def topology_section(args, hg, sources, kinds, cfg, mcc, stream):
    """The same queries through the topology-driven Iterate (every invocation
    visits all vertices, ReduceAndReturn Any(changed)): per-query time and
    work against the data-driven loop, results compared bit for bit."""
    import torch
    from paper_1607_05707_amd import irgl
    dev = hg.row_ptr.device
    tcfg = dict(cfg, mode=irgl.IRGL_MODE_TOPOLOGY)
    out_d = torch.empty(hg.n, dtype=torch.int32, device=dev)
    out_t = torch.empty(hg.n, dtype=torch.int32, device=dev)
    stats = irgl.stats_tensor(dev)
    fns = {0: irgl.irgl_bfs, 1: irgl.irgl_sssp}
    res = {"sources": len(sources), "matches_data_driven": True}
    for k in kinds:
        ws_d = irgl.workspace(hg, k, False, cfg)
        ws_t = irgl.workspace(hg, k, False, tcfg)
        tot_ms, iters, edges, d_iters, d_edges = 0.0, 0, 0, 0, 0
        for s in sources:
            fns[k](hg, s, out_d, None, ws_d, stream, stats, cfg)
            st = irgl.read_stats(stats)
            d_iters += st["iterations"]
            d_edges += st["edges"]
            fns[k](hg, s, out_t, None, ws_t, stream, None, tcfg)  # warm
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fns[k](hg, s, out_t, None, ws_t, stream, stats, tcfg)
            b.record(stream)
            torch.cuda.synchronize()
            tot_ms += a.elapsed_time(b)
            st = irgl.read_stats(stats)
            if st["status"] != 0:
                raise SystemExit(f"topology-driven kind {k} from {s} failed: {irgl.irgl_status_string(st['status'])}")
            iters += st["iterations"]
            edges += st["edges"]
            res["matches_data_driven"] &= bool(torch.equal(out_d, out_t))
        nq = len(sources)
        res[{0: "bfs", 1: "sssp"}[k]] = {
            "avg_query_us": round(1e3 * tot_ms / nq, 1),
            "gteps": round(sum(mcc[s] for s in sources) / (tot_ms / 1e3) / 1e9, 3),
            "invocations": round(iters / nq, 1), "edges_scanned": int(edges / nq),
            "data_driven_invocations": round(d_iters / nq, 1), "data_driven_edges_scanned": int(d_edges / nq)}
    log(f"topology-driven {res}")
    return res


def mst_section(hg, stream):
    """Boruvka minimum spanning forest of the same graph (the Atomic
    construct's workload) with each compilation of its atomic section: time,
    rounds, scanned entries; the three forests must be identical."""
    import torch
    from paper_1607_05707_amd import irgl
    dev = hg.row_ptr.device
    res = {"graph": "the bench graph (caller's labelling)", "identical_forests": True}
    ws = torch.empty(irgl.irgl_mst_workspace_bytes(hg), dtype=torch.uint8, device=dev)
    ref = None
    for name, lock in (("packed", irgl.IRGL_LOCK_PACKED), ("spin", irgl.IRGL_LOCK_SPIN),
                       ("ticket", irgl.IRGL_LOCK_TICKET)):
        weight = torch.zeros(1, dtype=torch.int64, device=dev)
        comp = torch.empty(hg.n, dtype=torch.int32, device=dev)
        forest = torch.empty(int(hg.col.numel()), dtype=torch.uint8, device=dev)
        stats = irgl.stats_tensor(dev)
        cfg = {"lock": lock}
        irgl.irgl_mst(hg, weight, comp, forest, ws, stream, stats, cfg)  # warm
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        irgl.irgl_mst(hg, weight, comp, forest, ws, stream, stats, cfg)
        b.record(stream)
        torch.cuda.synchronize()
        st = irgl.read_stats(stats)
        if st["status"] != 0:
            raise SystemExit(f"mst ({name}) failed: {irgl.irgl_status_string(st['status'])}")
        out = (int(weight.item()), comp.clone(), forest.clone())
        if ref is None:
            ref = out
        else:
            res["identical_forests"] &= out[0] == ref[0] and bool(torch.equal(out[1], ref[1])) and \
                bool(torch.equal(out[2], ref[2]))
        res[name] = {"ms": round(a.elapsed_time(b), 3), "rounds": st["iterations"], "edges_scanned": st["edges"]}
    res["weight"] = ref[0]
    res["forest_edges"] = int(ref[2].sum().item()) // 2
    log(f"mst {res}")
    return res


def batched_section(args, dev):
    """The batched workload (seed 256: uniform graphs of uneven size, BFS/SSSP
    alternating, plus R-MAT scale 20 with 64 BFS sources) in ONE persistent
    launch, against the same queries each in its own launch ("plain")."""
    import torch
    from paper_1607_05707_amd import autotune, irgl
    t0 = time.perf_counter()
    keep, tasks = autotune.batch_tasks(256, args.batch_count, dev)
    torch.cuda.synchronize()
    log(f"batched workload: {len(tasks)} tasks, generated in {time.perf_counter() - t0:.1f}s")
    # numerator per task: m_cc from an untimed BFS from the same source
    mcc = []
    for hg, kind, src in tasks:
        _, _, st = irgl.query(hg, 0, src)
        mcc.append(st["frontier_edges"])
    cfg = autotune.load("batch")
    t_batch = autotune.time_batch(tasks, cfg, reps=2)
    # plain: one launch per query, back to back on one stream
    outs = {}
    wss = {}
    for hg, kind, src in tasks:
        key = (id(hg), kind)
        if key not in wss:
            wss[key] = irgl.workspace(hg, kind)
            outs[id(hg)] = torch.empty(hg.n, dtype=torch.int32, device=dev)
    best_plain = float("inf")
    best_dev = float("inf")
    stream = torch.cuda.current_stream(dev)
    for _ in range(2):
        torch.cuda.synchronize()
        evs = []
        t0 = time.perf_counter()
        for hg, kind, src in tasks:
            fn = irgl.irgl_bfs if kind == 0 else irgl.irgl_sssp
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn(hg, src, outs[id(hg)], None, wss[(id(hg), kind)], stream)
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        best_plain = min(best_plain, time.perf_counter() - t0)
        best_dev = min(best_dev, sum(a.elapsed_time(b) for a, b in evs) / 1e3)
    total = float(sum(mcc))
    log(f"batched {t_batch * 1e3:.1f} ms vs plain {best_plain * 1e3:.1f} ms "
        f"(device time of the plain launches {best_dev * 1e3:.1f} ms)")
    return {"tasks": len(tasks), "config": cfg, "batched_ms": round(t_batch * 1e3, 2),
            "plain_ms": round(best_plain * 1e3, 2), "speedup": round(best_plain / t_batch, 3),
            "plain_device_ms": round(best_dev * 1e3, 2), "speedup_vs_device": round(best_dev / t_batch, 3),
            "batched_gteps": round(total / t_batch / 1e9, 3), "plain_gteps": round(total / best_plain / 1e9, 3)}


def served_section(args, dev):
    """Continuous batching over the eight resident graphs.  p50/p99 latency
    and throughput, served against plain FIFO single launches: a Poisson
    stream at fractions of the plain capacity, a saturating burst (every
    query arrives at once: throughput of each form when never idle), and the
    same burst under a small per-query state budget (admission by memory)."""
    import numpy as np
    from paper_1607_05707_amd import autotune, serve
    t0 = time.perf_counter()
    graphs = serve.resident_set("full", dev)
    log(f"served set resident in {time.perf_counter() - t0:.1f}s")
    cap_q = serve.query_stream(graphs, 200, 6)
    capacity = serve.measure_capacity(graphs, cap_q)
    cfg = autotune.load("serve")
    budget = 4 << 30
    sweep = {}
    for frac in [float(x) for x in args.serve_lambdas.split(",")]:
        queries = serve.query_stream(graphs, args.serve_queries, 5)
        arr = serve.poisson_arrivals(len(queries), frac * capacity, 12)
        info = {}
        lat_s, wall_s, _, rej = serve.run_served(graphs, queries, arr, budget, cfg=cfg, info=info)
        lat_p, wall_p = serve.run_plain(graphs, queries, arr)
        sweep[str(frac)] = {"served": serve.summarize(lat_s, wall_s), "plain": serve.summarize(lat_p, wall_p),
                            "rejected": rej, **info}
        log(f"served lambda={frac}: {sweep[str(frac)]}")
    queries = serve.query_stream(graphs, args.serve_burst, 7)
    burst = np.zeros(len(queries))
    info = {}
    lat_s, wall_s, _, rej = serve.run_served(graphs, queries, burst, budget, cfg=cfg, info=info)
    lat_p, wall_p = serve.run_plain(graphs, queries, burst)
    saturating = {"queries": len(queries), "served": serve.summarize(lat_s, wall_s),
                  "plain": serve.summarize(lat_p, wall_p), "rejected": rej, **info}
    saturating["qps_ratio"] = round(saturating["served"]["qps"] / saturating["plain"]["qps"], 3)
    log(f"served saturating burst: {saturating}")
    small_budget = args.serve_small_budget_mb << 20
    info = {}
    lat_m, wall_m, _, rej_m = serve.run_served(graphs, queries, burst, small_budget, cfg=cfg, info=info)
    memory_bound = {"budget_mb": args.serve_small_budget_mb, "served": serve.summarize(lat_m, wall_m),
                    "rejected": rej_m, **info}
    log(f"served under a {args.serve_small_budget_mb} MiB state budget: {memory_bound}")
    return {"graphs": len(graphs), "config": cfg, "plain_capacity_qps": round(capacity, 1), "budget_gb": 4,
            "queries_per_lambda": args.serve_queries, "lambda_sweep": sweep, "saturating": saturating,
            "memory_bound": memory_bound}


def level_section(dev, stream, name, reps=2):
    """Barrier-bound workloads: one BFS and one SSSP from source 0, time per
    invocation (the outlined loop's cost per level) and per query."""
    import torch
    from paper_1607_05707_amd import irgl
    from paper_1607_05707_amd.workloads import make_workload
    g = make_workload(name, dev, 1)
    hg = irgl.upload(g, reorder=True)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    stats = irgl.stats_tensor(dev)
    res = {"n": g.n, "m": g.m}
    for k, fn in ((0, irgl.irgl_bfs), (1, irgl.irgl_sssp)):
        ws = irgl.workspace(hg, k)
        fn(hg, 0, out, None, ws, stream, stats)  # warm
        best = float("inf")
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn(hg, 0, out, None, ws, stream, stats)
            b.record(stream)
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        st = irgl.read_stats(stats)
        if st["status"] != 0:
            raise SystemExit(f"{name} kind {k} failed: {irgl.irgl_status_string(st['status'])}")
        res[["bfs", "sssp"][k]] = {"query_us": round(best * 1e3, 1), "invocations": st["iterations"],
                                   "us_per_invocation": round(best * 1e3 / max(1, st["iterations"]), 2)}
    log(f"{name}: {res}")
    del hg
    return res


def road_section(dev, stream, reps=2):
    """The road-like 4096 x 4096 grid with its long edges: BFS and SSSP from
    its 9 sources, GTEPS and the fraction of the HBM roofline per kind."""
    import torch
    from paper_1607_05707_amd import irgl
    from paper_1607_05707_amd.workloads import make_workload
    g = make_workload("road4096", dev, 9)
    hg = irgl.upload(g, reorder=True)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    stats = irgl.stats_tensor(dev)
    res = {"n": g.n, "m": g.m, "sources": len(g.sources)}
    mcc, reached = {}, {}
    ws0 = irgl.workspace(hg, 0)
    for s in g.sources:
        irgl.irgl_bfs(hg, s, out, None, ws0, stream, stats)
        st = irgl.read_stats(stats)
        mcc[s], reached[s] = st["frontier_edges"], st["items"]
    for k, fn in ((0, irgl.irgl_bfs), (1, irgl.irgl_sssp)):
        ws = irgl.workspace(hg, k)
        tot = 0.0
        for s in g.sources:
            fn(hg, s, out, None, ws, stream, stats)  # warm
            best = float("inf")
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn(hg, s, out, None, ws, stream, stats)
                b.record(stream)
                torch.cuda.synchronize()
                best = min(best, a.elapsed_time(b))
            st = irgl.read_stats(stats)
            if st["status"] != 0:
                raise SystemExit(f"road4096 kind {k} from {s} failed: {irgl.irgl_status_string(st['status'])}")
            tot += best
        nq = len(g.sources)
        alg = sum(alg_bytes(k, g.n, reached[s], mcc[s]) for s in g.sources) / nq
        avg_ms = tot / nq
        res[["bfs", "sssp"][k]] = {"avg_query_us": round(avg_ms * 1e3, 1),
                                   "gteps": round(sum(mcc.values()) / (tot / 1e3) / 1e9, 3),
                                   "alg_bytes_per_query": int(alg),
                                   "roofline_frac": round(alg / (avg_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
    log(f"road4096: {res}")
    del hg
    return res


def dmr_section(args, dev):
    """Delaunay mesh refinement (the Exclusive construct's workload, one
    cooperative launch running the DMR pipe) of a random-square mesh: time
    per refinement, points inserted and triangles made per second, and the
    oracle's validity check of one refined mesh."""
    import torch
    from paper_1607_05707_amd import irgl, meshgen
    t0 = time.perf_counter()
    m = meshgen.random_square(args.dmr_points, 42)
    log(f"dmr mesh {m.name}: {m.npts} points, {m.ntri} triangles, generated in {time.perf_counter() - t0:.1f}s")
    best, st, dm = float("inf"), None, None
    for _ in range(args.dmr_reps):
        dm = irgl.DeviceMesh.from_host(m, dev)
        ws = torch.empty(irgl.irgl_dmr_workspace_bytes(dm), dtype=torch.uint8, device=dev)
        stats = torch.zeros(irgl.DMR_STATS_BYTES, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        irgl.irgl_dmr_refine(dm, ws, None, None, stats)
        b.record()
        torch.cuda.synchronize()
        st = irgl.read_dmr_stats(stats)
        if st["status"] != 0:
            raise SystemExit(f"dmr failed: {irgl.irgl_status_string(st['status'])}")
        best = min(best, a.elapsed_time(b))
    res = {"mesh": m.name, "input_points": m.npts, "input_triangles": m.ntri, "min_angle": 30.0,
           "ms": round(best, 2), "points": st["npts"], "triangles": st["ntri"],
           "inserted": st["inserted"], "splits": st["splits"], "invocations": st["invocations"],
           "rounds": st["rounds"], "refined": st["refined"], "conflicts": st["conflicts"],
           "max_cavity": st["max_cavity"], "final_bad": st["final_bad"],
           "mpoints_per_s": round((st["npts"] - m.npts) / (best / 1e3) / 1e6, 2),
           "mtriangles_per_s": round(st["ntri"] / (best / 1e3) / 1e6, 2)}
    if not args.no_dmr_check:
        from oracle import mesh as om
        t0 = time.perf_counter()
        chk = om.check_mesh(dm.pts[:st["npts"]].cpu().numpy(), dm.tri[:st["ntri"]].cpu().numpy(),
                            dm.nbr[:st["ntri"]].cpu().numpy(), input_pts=m.input_pts, min_angle=30.0)
        res["oracle_check"] = {"valid": True, "min_angle": round(chk["min_angle"], 4),
                               "seconds": round(time.perf_counter() - t0, 1)}
    log(f"dmr {res}")
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--kinds", default="bfs,sssp")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--t-wave", type=int, default=0)
    ap.add_argument("--t-block", type=int, default=0)
    ap.add_argument("--t-grid", type=int, default=0)
    ap.add_argument("--t-bitmap", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--mode", default="persistent", choices=["persistent", "hostloop"])
    ap.add_argument("--reorder", type=int, default=1, choices=[0, 1],
                    help="1 (default): upload through irgl_graph_upload_reordered (degree-sorted "
                         "relabelling, one-time, results under caller ids); 0: plain upload")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-topology", action="store_true")
    ap.add_argument("--no-mst", action="store_true")
    ap.add_argument("--topology-sources", type=int, default=8)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-queries", type=int, default=400, help="queries per point of the lambda sweep")
    ap.add_argument("--serve-lambdas", default="0.25,0.5,0.8,0.95")
    ap.add_argument("--serve-burst", type=int, default=600)
    ap.add_argument("--serve-small-budget-mb", type=int, default=96)
    ap.add_argument("--no-levels", action="store_true", help="skip the grid64 / road4096 legs")
    ap.add_argument("--no-dmr", action="store_true", help="skip the mesh-refinement leg")
    ap.add_argument("--no-dmr-check", action="store_true", help="skip the oracle check of the refined mesh")
    ap.add_argument("--dmr-points", type=int, default=1000000)
    ap.add_argument("--dmr-reps", type=int, default=3)
    ap.add_argument("--calibrate-mb", type=int, default=0,
                    help="first copy this many MiB device to device once (a copy of known traffic that "
                         "scales hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(batched and served queries would shard by replicating the graphs and "
              "routing each query to one GPU). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from paper_1607_05707_amd import irgl
    from paper_1607_05707_amd.workloads import make_workload

    dev = torch.device("cuda:0")
    if args.calibrate_mb > 0:
        a = torch.ones(args.calibrate_mb << 18, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_mb} MiB read + {args.calibrate_mb} MiB written")
        del a, b
    kinds = [{"bfs": 0, "sssp": 1}[k] for k in args.kinds.split(",")]
    t0 = time.perf_counter()
    g = make_workload(args.workload, dev, args.sources)
    torch.cuda.synchronize()
    log(f"generated {g.name}: n={g.n} m={g.m} sources={len(g.sources)} in {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    hg = irgl.upload(g, reorder=bool(args.reorder))
    torch.cuda.synchronize()
    upload_ms = 1e3 * (time.perf_counter() - t_up)
    log(f"upload ({'degree-sorted relabelling' if args.reorder else 'caller ids'}): {upload_ms:.1f} ms (untimed)")
    cfg = {"block": args.block, "t_wave": args.t_wave, "t_block": args.t_block, "t_grid": args.t_grid,
           "t_bitmap": args.t_bitmap, "grid": args.grid,
           "mode": 1 if args.mode == "hostloop" else 0}
    sources = list(g.sources)

    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = {k: irgl.workspace(hg, k, False, cfg) for k in kinds}
    stats = irgl.stats_tensor(dev)
    stream = torch.cuda.current_stream()
    fns = {0: irgl.irgl_bfs, 1: irgl.irgl_sssp}

    # per-source numerator m_cc and reached count from one BFS each (untimed)
    mcc, reached, gpu_results = {}, {}, {}
    blocks = {}  # workgroup size each kind resolved to
    n_check = min(len(sources), 2)
    for i, s in enumerate(sources):
        irgl.irgl_bfs(hg, s, out, None, ws[kinds[0]] if 0 in ws else irgl.workspace(hg, 0), stream,
                      stats, cfg)
        st = irgl.read_stats(stats)
        if st["status"] != 0:
            raise SystemExit(f"BFS from {s} failed: {irgl.irgl_status_string(st['status'])}")
        mcc[s] = st["frontier_edges"]
        reached[s] = st["items"]
        blocks[0] = st["block"]
        if i < n_check:
            lv = irgl.as_u32_numpy(out).copy()
            d = None
            if 1 in kinds:
                irgl.irgl_sssp(hg, s, out, None, ws[1], stream, stats, cfg)
                d = irgl.as_u32_numpy(out).copy()
                blocks[1] = irgl.read_stats(stats)["block"]
            gpu_results[s] = (lv, d)
    log(f"m_cc: mean {sum(mcc.values()) / len(mcc):.0f} over {len(mcc)} sources")

    # every timed query writes its own statistics block, so that a failure of
    # any one of them (not only the last) fails the bench
    nq_step = len(sources) * len(kinds)
    qstats = torch.zeros((args.steps * nq_step, irgl.STATS_BYTES), dtype=torch.uint8, device=dev)

    # host-side objects of the timed loop made once: the configuration as the
    # ABI struct, the stats views and the event pairs
    cfg_c = irgl.make_config(cfg)
    qviews = [qstats[i] for i in range(qstats.shape[0])]
    evpool = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(qstats.shape[0])]

    def one_step(record, step=0):
        q = step * nq_step
        for s in sources:
            for k in kinds:
                if record is not None:
                    a, b = evpool[q]
                    a.record(stream)
                    fns[k](hg, s, out, None, ws[k], stream, qviews[q], cfg_c)
                    b.record(stream)
                    record.append((k, s, a, b, q))
                    q += 1
                else:
                    fns[k](hg, s, out, None, ws[k], stream, None, cfg_c)

    for _ in range(args.warmup):
        one_step(None)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    events = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        one_step(events, i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    names_k = {0: "bfs", 1: "sssp"}
    all_stats = irgl.read_stats_array(qstats)
    bad = [(names_k[k], s, st["status"]) for (k, s, _, _, q), st in zip(events, all_stats) if st["status"] != 0]
    if bad:
        raise SystemExit(f"{len(bad)} timed queries failed, first: {bad[0][0]} from {bad[0][1]}: "
                         f"{irgl.irgl_status_string(bad[0][2])}")
    per_kind_ms = {k: [] for k in kinds}
    per_kind_edges = {k: 0 for k in kinds}
    for (k, s, a, b, q), st in zip(events, all_stats):
        per_kind_ms[k].append(a.elapsed_time(b))
        per_kind_edges[k] += st["edges"]
    teps_edges = args.steps * sum(mcc[s] for s in sources) * len(kinds)
    value = teps_edges / elapsed / 1e9

    kind_summary = {}
    for k in kinds:
        ms = per_kind_ms[k]
        tot_ms = sum(ms)
        edges = args.steps * sum(mcc[s] for s in sources)
        bytes_per_query = sum(alg_bytes(k, g.n, reached[s], mcc[s]) for s in sources) / len(sources)
        avg_ms = tot_ms / len(ms)
        kind_summary[k] = {
            "gteps": round(edges / (tot_ms / 1e3) / 1e9, 3),
            "avg_query_us": round(avg_ms * 1e3, 1),
            "alg_bytes_per_query": int(bytes_per_query),
            "alg_gbs": round(bytes_per_query / (avg_ms / 1e3) / 1e9, 1),
            # CSR entries the kernel scanned per entry of the reached component
            "scans_per_edge": round(per_kind_edges[k] / edges, 3),
            "total_ms": tot_ms,
        }
    # measured HBM bytes per launch of each kind's kernel (rocprofv3
    # FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), only while the HIP
    # sources are the ones the counters were taken on.  BFS algorithmic
    # bytes count a top-down traversal; bottom-up invocations scan fewer
    # entries, so its measured traffic can sit below them.
    from paper_1607_05707_amd import profiling
    kernel_of = {k: f"persistent_kernel<{blocks[k]}, irgl::{['BfsOp', 'SsspOp'][k]}>" for k in kinds}
    traffic_of = {}
    for k in kinds:
        rec = profiling.load_traffic(os.path.join(ROOT, "profiles", f"traffic_{args.workload}_{names_k[k]}.json"))
        traffic_of[k] = int(rec["traffic_bytes_per_launch"]) if rec and rec.get("kernel") == kernel_of[k] else None
        kind_summary[k]["roofline_frac"] = round(kind_summary[k]["alg_gbs"] / PEAK_HBM_GBS, 4)
        kind_summary[k]["traffic_bytes_per_launch"] = traffic_of[k]
        kind_summary[k]["traffic_over_alg"] = (round(traffic_of[k] / kind_summary[k]["alg_bytes_per_query"], 3)
                                               if traffic_of[k] else None)
    dom = max(kinds, key=lambda k: kind_summary[k]["total_ms"])
    ks = kind_summary[dom]
    kname = kernel_of[dom]
    traffic = traffic_of[dom]
    roofline = {
        "bound": "hbm",
        "achieved": ks["alg_gbs"],
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(ks["alg_gbs"] / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch",
        "alg_bytes_per_launch": ks["alg_bytes_per_query"],
        "kernel": f"{kname} (timed with its init fill and the scatter of results to caller ids)",
    }

    mst = None
    if not args.no_mst:
        mst = mst_section(hg, stream)

    topology = None
    if not args.no_topology:
        topology = topology_section(args, hg, sources[:args.topology_sources], kinds, cfg, mcc, stream)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu, parity = cpu_baseline(g, sources, args.cpu_budget, gpu_results)

    batched = None
    if not args.no_batched:
        batched = batched_section(args, dev)
    served = None
    if not args.no_served:
        served = served_section(args, dev)

    levels = None
    if not args.no_levels:
        levels = {"grid64": level_section(dev, stream, "grid64"),
                  "road4096_nolong": level_section(dev, stream, "road4096_nolong", reps=1),
                  "road4096": road_section(dev, stream)}

    dmr = None
    if not args.no_dmr:
        dmr = dmr_section(args, dev)

    names = {0: "bfs", 1: "sssp"}
    line = {
        "metric": "GTEPS BFS/SSSP on RMAT-22, batched vs plain; HBM GB/s; p99 query latency",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{g.name}: plain BFS+SSSP, one launch per query, {len(sources)} sources",
            "n": g.n,
            "m": g.m,
            "sources": len(sources),
            "queries_per_step": len(sources) * len(kinds),
            "mode": args.mode,
            "block": {names[k]: blocks[k] for k in kinds},
            "upload": "degree-sorted relabelling" if args.reorder else "caller ids",
            "upload_ms_untimed": round(upload_ms, 1),
        },
        "per_kind": {names[k]: {kk: vv for kk, vv in kind_summary[k].items() if kk != "total_ms"}
                     for k in kinds},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "batched": batched,
        "served": served,
        "topology": topology,
        "mst": mst,
        "levels": levels,
        "dmr": dmr,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
