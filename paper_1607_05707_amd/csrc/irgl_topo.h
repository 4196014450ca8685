// Topology-driven Iterate: the paper's other loop form (Table 1: a ForAll
// over every node of the graph whose kernel returns a reduced boolean through
// ReduceAndReturn; Iterate While Any / Until All re-invokes it until the
// reduction says nothing changed).  No worklists: every invocation visits all
// n vertices with the same nested edge parallelism as the data-driven loop
// (identity worklist), and the outlined loop runs in one cooperative launch
// with the grid barrier between invocations.
//
// ReduceAndReturn is compiled the way Section 3 describes its cheaper form:
// every thread holds its own value, the workgroup combines them with one
// barrier-OR, and only one atomic per workgroup reaches the global word
// (Any: set when some thread's value is true; All: set when some thread's
// value is false).  The words rotate over three invocations like the
// worklist counters, so none needs a second barrier to be cleared.
#pragma once

#include "irgl_query.h"

namespace irgl {

// Block-aggregated ReduceAndReturn.  All threads of the workgroup call it.
// After the next team barrier the invocation's result is
// Any: *word != 0; All: *word == 0.
__device__ __forceinline__ void reduce_and_return(bool value, bool all, uint32_t *word) {
    const bool mark = all ? !value : value;
    if (__syncthreads_or(mark) && threadIdx.x == 0) atomicOr(word, 1u);
}

// BFS, topology-driven: invocation r expands every vertex labelled r and
// labels its unlabelled neighbours r + 1.  Every writer of a label in one
// invocation writes the same value, so a plain store is a correct claim (no
// atomics); a parent written by a racing writer is still a vertex of level r.
// `wins` counts the labels this lane wrote (the invocation's "changed").
struct BfsTopoOp {
    static constexpr bool kPush = false;
    static constexpr bool kFar = false;
    static constexpr int kU = 4;
    static constexpr int kMinWaves = 1;
    uint32_t *level;
    int32_t *parent;
    uint32_t cur;
    const int32_t *perm;  // relabelled graph: parents are stored as caller ids
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return level[v]; }
    __device__ __forceinline__ bool active(uint32_t lv) const { return lv == cur; }
    __device__ __forceinline__ void relax(const int (&)[kU], const int (&d)[kU], const int (&sv)[kU],
                                          const uint32_t (&)[kU], bool (&act)[kU], bool (&)[kU], uint32_t &,
                                          uint32_t &tries, uint32_t &wins) const {
        uint32_t lv[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) lv[k] = act[k] ? level[d[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const bool label = act[k] && lv[k] == kInf;
            tries += label ? 1u : 0u;
            wins += label ? 1u : 0u;
            if (label) {
                level[d[k]] = cur + 1;
                if (parent) parent[d[k]] = perm ? perm[sv[k]] : sv[k];
            }
            act[k] = false;
        }
    }
};

// SSSP, topology-driven (Bellman-Ford): every invocation relaxes the edges of
// every reached vertex with atomicMin; a relaxation that lowers a distance
// counts as a change.  A plain (possibly stale) probe of dist filters first:
// a stale value is only ever larger, so it lets more through, never fewer.
struct SsspTopoOp {
    static constexpr bool kPush = false;
    static constexpr bool kFar = false;
    static constexpr int kU = 2;
    static constexpr int kMinWaves = 5;
    uint32_t *dist;
    const uint32_t *w;
    Ctrl *ctrl;
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return dist[v]; }
    __device__ __forceinline__ bool active(uint32_t dv) const { return dv != kInf; }
    __device__ __forceinline__ void relax(const int (&e)[kU], const int (&d)[kU], const int (&)[kU],
                                          const uint32_t (&dv)[kU], bool (&act)[kU], bool (&)[kU], uint32_t &,
                                          uint32_t &tries, uint32_t &wins) const {
        uint32_t nd[kU], cur[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) nd[k] = act[k] ? w[e[k]] : 0u;
        bool ovf = false;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const uint32_t s = dv[k] + nd[k];
            const bool bad = act[k] && (s < dv[k] || s == kInf);  // does not fit below INF
            ovf |= bad;
            act[k] = act[k] && !bad;
            nd[k] = s;
        }
        if (ovf) set_error(ctrl, kErrOverflow, false);
#pragma unroll
        for (int k = 0; k < kU; ++k) cur[k] = act[k] ? dist[d[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const bool try_it = act[k] && nd[k] < cur[k];
            tries += try_it ? 1u : 0u;
            const bool won = try_it && nd[k] < atomicMin(&dist[d[k]], nd[k]);
            wins += won ? 1u : 0u;
            act[k] = false;
        }
    }
};

template <class Op> struct TopoOf;
template <> struct TopoOf<BfsOp> { using type = BfsTopoOp; };
template <> struct TopoOf<SsspOp> { using type = SsspTopoOp; };

template <class Op>
__device__ __forceinline__ Op make_topo_op(const Params &p, uint32_t it);

template <>
__device__ __forceinline__ BfsTopoOp make_topo_op<BfsTopoOp>(const Params &p, uint32_t it) {
    return BfsTopoOp{p.val, p.parent, it, p.perm};
}

template <>
__device__ __forceinline__ SsspTopoOp make_topo_op<SsspTopoOp>(const Params &p, uint32_t) {
    return SsspTopoOp{p.val, p.w, p.ctrl};
}

// The outlined topology-driven loop run by the team.  Invocation `it`:
// ForAll over all vertices (phase A, grid-tier phase B when vertices were
// deferred), then ReduceAndReturn of "this thread changed something", then a
// team barrier; the loop continues while the reduction says something
// changed (Any(changed) true, or All(unchanged) false).  A round without
// deferred vertices has one barrier, otherwise two.
template <int B, class Op>
__device__ __forceinline__ LoopResult run_topology(const Params &p, Smem<B> &sm, Team tm, BarrierState &bs) {
    const int wid = threadIdx.x / kWave;
    Ctrl *ctrl = p.ctrl;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{nullptr, nullptr, 0u, ctrl, nullptr},
               Sink{nullptr, nullptr, 0u, ctrl, nullptr}, kInf};
    LoopResult r{0u, 0ull, 0ull, 0u, 0ull, 0u};
    const bool lead = tm.id == 0 && threadIdx.x == 0;
    const bool all = p.reduce_all != 0;
    const uint32_t n = static_cast<uint32_t>(p.n);
    uint32_t it = 0;
    for (;; ++it) {
        if (it >= p.max_iter) {
            if (lead) set_error(ctrl, kErrIterLimit, false);
            break;
        }
        if (lead) {
            // red[(it + 1) % 3] was last read after invocation it - 2, before
            // invocation it - 1's barrier; it is next written in invocation it + 1
            store_agent(&ctrl->red[(it + 1) % 3], 0u);
            store_agent(&ctrl->tile[(it + 2) % 3], 0u);
            __hip_atomic_store(&ctrl->hub[(it + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        r.items += n;
        const Op op = make_topo_op<Op>(p, it);
        unsigned long long *hub_ctr = &ctrl->hub[it % 3];
        uint32_t *red = &ctrl->red[it % 3];
        pu.wins = 0;
        expand<B, Op>(nullptr, n, n, p.row_ptr, p.col, op, sm, pu, p.t_wave, p.t_block, p.t_grid, p.hub_v,
                      p.hub_base, p.hub_cap, hub_ctr, r.edges, tm, &ctrl->tile[it % 3]);
        // ReduceAndReturn of phase A: Any(changed) or All(unchanged), at most
        // one atomic per workgroup, complete once the barrier has passed
        reduce_and_return(all ? pu.wins == 0u : pu.wins != 0u, all, red);
        if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
        if (p.t_grid > 0) {
            uint32_t nh, nchunks;
            hub_counts(__hip_atomic_load(hub_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), p.hub_cap, nh,
                       nchunks);
            if (nh > 0) {  // uniform: read after the barrier
                expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, op, sm, pu, tm);
                // the grid-tier phase adds its own changes to the same word
                reduce_and_return(all ? pu.wins == 0u : pu.wins != 0u, all, red);
                if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
            }
        }
        const uint32_t word = load_agent(red);
        // the invocation's return value: Any(changed) = some workgroup marked
        // a change; All(unchanged) = no workgroup marked an unchanged-false
        const bool result = all ? word == 0u : word != 0u;
        const bool again = all ? !result : result;  // Until All / While Any
        if (!again) {
            ++it;
            break;
        }
    }
    r.iterations = it;
    r.fedges = r.edges;  // every scanned edge belongs to a visited vertex
    return r;
}

// One topology-driven query per cooperative launch.
template <int B, class Op>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(fit_waves<B, Op::kMinWaves>()))) void topology_kernel(
    Params p) {
    __shared__ Smem<B> sm;
    const Team tm = whole_grid();
    BarrierState bs = make_barrier_state(p.wd_ticks, p.barrier);
    const LoopResult r = run_topology<B, Op>(p, sm, tm, bs);
    finish_query<B>(p, r, tm);
}

}  // namespace irgl
