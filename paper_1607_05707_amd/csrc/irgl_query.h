// Query-level kernels: initialisation, the visited-bitmap refresh, the
// outlined persistent Iterate loop, the un-outlined per-invocation kernels,
// the SSSP parent pass and the on-device CSR validation.
#pragma once

#include "irgl_expand.h"

namespace irgl {

// ---------------------------------------------------------------------------
// Initialisation: val = INF except val[src] = 0; parent = -1 except
// parent[src] = src; stamps = INF; SSSP shadow = dist; far flags = 0;
// bitmap = {src}; in = [src];
// counters and stats cleared.
// ---------------------------------------------------------------------------
// Per-query fill, grid-strided over the team.
__device__ __forceinline__ void init_arrays(const Params &p, int with_stamp, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t i = tm.id * blockDim.x + threadIdx.x; i < n; i += tm.size * blockDim.x) {
        const bool s = static_cast<int>(i) == p.src;
        p.val[i] = s ? 0u : kInf;
        if (p.parent) p.parent[i] = s ? p.src_orig : -1;
        if (with_stamp) {
            p.stamp[i] = kInf;
            if (p.shadow16) reinterpret_cast<uint16_t *>(p.shadow)[i] = s ? 0 : 0xFFFF;
            else p.shadow[i] = s ? 0u : kInf;
            p.far_flag[i] = 0u;
            if (p.expd) p.expd[i] = kInf;
            if (p.hstamp) p.hstamp[i] = kInf;
        }
        if (p.visited && (i & 31u) == 0u)
            p.visited[i >> 5] = (static_cast<uint32_t>(p.src) >> 5 == i >> 5)
                                    ? (1u << (p.src & 31)) : 0u;
    }
}

// Per-query control-block reset (one thread).  Barrier words are reset only
// by a fresh launch (reset_barrier): a batched team keeps its barrier
// counters, which only grow, across the queries it runs.
__device__ __forceinline__ void init_control(const Params &p, bool reset_barrier) {
        Ctrl *c = p.ctrl;
        c->cnt[0] = 1;
        c->cnt[1] = 0;
        c->cnt[2] = 0;
        for (int k = 0; k < 3; ++k) {
            c->tile[k] = 0;
            c->red[k] = 0;
            c->hub[k] = 0;
            c->far_cnt[k] = 0;
            c->far_min[k] = kInf;
            c->hcnt[k] = 0;
            c->hsum[k] = 0;
            c->hmin[k] = kInf;
            c->hbig[k] = 0;
        }
        if (reset_barrier) reset_barrier_words(c);
        c->error = 0;
        c->fatal = 0;
        c->done = 0;
        c->iterations = 0;
        c->max_frontier = 0;
        c->items = 0;
        c->edges = 0;
        c->fedges = 0;
        c->pulls = 0;
        c->mf[0] = static_cast<unsigned long long>(p.row_ptr[p.src + 1] - p.row_ptr[p.src]);
        c->mf[1] = 0;
        c->mf[2] = 0;
        c->bu_scan = 0;
        p.wl0[0] = p.src;
}

__global__ void init_kernel(Params p, int with_stamp) {
    init_arrays(p, with_stamp, whole_grid());
    if (blockIdx.x == 0 && threadIdx.x == 0) init_control(p, true);
}

// The operator of invocation `it`.  SSSP: `bucket` is the number of
// threshold raises so far; `heavy` selects the heavy pass of a split graph
// (heavy ranges, no pop-time skip or listing).
template <class Op>
__device__ __forceinline__ Op make_op(const Params &p, uint32_t it, uint32_t thresh, uint32_t bucket = 0,
                                      bool heavy = false);

template <>
__device__ __forceinline__ SsspOp make_op<SsspOp>(const Params &p, uint32_t it, uint32_t thresh, uint32_t bucket,
                                                  bool heavy) {
    SsspOp op{p.val, p.w, p.stamp, p.far_flag, thresh, it, p.ctrl, p.visited, p.shadow};
    op.shadow16 = p.shadow16;
    // without a threshold (the bucketing has ended) an expansion relaxes the
    // whole row and lists nothing: every vertex listed before has its heavy
    // pass in the transfer that ended the bucketing, so no heavy pass (and
    // no transfer invocation) is left
    const bool whole = !heavy && thresh == kInf;
    op.split = whole ? nullptr : p.split;
    op.expd = heavy ? nullptr : p.expd;
    op.hstamp = (heavy || whole || !p.split) ? nullptr : p.hstamp;
    op.bucket = bucket;
    op.heavy = heavy ? 1u : 0u;
    return op;
}

template <>
__device__ __forceinline__ BfsOp make_op<BfsOp>(const Params &p, uint32_t it, uint32_t, uint32_t, bool) {
    return BfsOp{p.val, p.parent, p.visited, it + 1, p.perm};
}

// Refresh a vertex bitmap from the value array: bit v = (val[v] < below).
// BFS: below = INF gives "visited"; SSSP: below = the threshold whose near
// phase has drained gives "settled" (final distance).  One ballot per 64
// consecutive vertices, coalesced reads, one plain word store per 32
// vertices.  Readers may see old or new words concurrently; both only ever
// mark vertices that qualify, so any mix is a valid filter.
__device__ __forceinline__ void refresh_bitmap(const Params &p, Team tm, uint32_t below) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    const uint32_t stride = tm.size * blockDim.x;
    for (uint32_t base = tm.id * blockDim.x; base < n; base += stride) {
        const uint32_t v = base + threadIdx.x;
        const bool vis = v < n && p.val[v] < below;
        const unsigned long long m = __ballot(vis);
        const int lane = lane_id();
        const uint32_t v0 = v - static_cast<uint32_t>(lane);  // first vertex of this wavefront
        if (lane == 0 && v0 < n) p.visited[v0 >> 5] = static_cast<uint32_t>(m);
        if (lane == 32 && v < n) p.visited[v >> 5] = static_cast<uint32_t>(m >> 32);
    }
}



// Write the control block's statistics to the caller's stats block.
__device__ __forceinline__ void publish_stats(const Params &p) {
    Ctrl *c = p.ctrl;
    if (!p.dstats) return;
    Stats *s = p.dstats;
    s->status = static_cast<int32_t>(load_agent(&c->error));
    s->iterations = c->iterations;
    s->items = c->items;
    s->edges = __hip_atomic_load(&c->edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s->max_frontier = c->max_frontier;
    s->grid = c->grid;
    s->block = c->block;
    s->heavy_pulls = c->pulls;
    s->frontier_edges = __hip_atomic_load(&c->fedges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum a per-thread counter over the workgroup and add it to *dst.
template <int B>
__device__ __forceinline__ void add_block_total(unsigned long long x, unsigned long long *dst) {
    __shared__ unsigned long long s_total;
    if (threadIdx.x == 0) s_total = 0;
    __syncthreads();
    atomicAdd(&s_total, x);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(dst, s_total);
}

// Trace of invocation `it` (only when a trace buffer is given), kTraceWords
// words at kTraceWords * it: start tick, incoming worklist size, edges
// scanned, vertices deferred to the grid tier, start tick of the grid-tier
// phase (0: none), claim atomics tried and won, then the largest and the
// summed per-workgroup busy ticks of the expansion phase and of the
// grid-tier phase (load balance), reserved.
constexpr uint32_t kTraceWords = 12;

__device__ __forceinline__ bool tracing(const Params &p, uint32_t it) {
    return kTraceWords * it + kTraceWords - 1 < p.trace_len;
}

__device__ __forceinline__ void trace_start(const Params &p, uint32_t it, uint32_t cnt_in) {
    unsigned long long *t = p.trace + kTraceWords * it;
    t[0] = wall_clock64();
    t[1] = cnt_in;
    for (uint32_t k = 2; k < kTraceWords; ++k) t[k] = 0;
}

// End of invocation `it`: this workgroup's edges and claim atomics.
template <class P>
__device__ __forceinline__ void trace_level(const Params &p, uint32_t it, unsigned long long edges,
                                            const unsigned long long *hub_ctr, Team tm, P &pu,
                                            unsigned long long busy_a = 0, unsigned long long busy_b = 0) {
    __shared__ unsigned long long s_sum[3];
    if (threadIdx.x < 3) s_sum[threadIdx.x] = 0;
    __syncthreads();
    if (edges) atomicAdd(&s_sum[0], edges);
    if (pu.tries) atomicAdd(&s_sum[1], static_cast<unsigned long long>(pu.tries));
    if (pu.wins) atomicAdd(&s_sum[2], static_cast<unsigned long long>(pu.wins));
    pu.tries = 0;
    pu.wins = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *t = p.trace + kTraceWords * it;
        atomicAdd(&t[2], s_sum[0]);
        atomicAdd(&t[5], s_sum[1]);
        atomicAdd(&t[6], s_sum[2]);
        atomicMax(&t[7], busy_a);
        atomicAdd(&t[8], busy_a);
        atomicMax(&t[9], busy_b);
        atomicAdd(&t[10], busy_b);
        if (tm.id == 0) t[3] = hub_ctr[0] >> 40;
    }
}

// Grid tier of invocation `it`: read the settled deferred-vertex counter.
__device__ __forceinline__ void hub_counts(unsigned long long hc, uint32_t hub_cap, uint32_t &nh,
                                           uint32_t &nchunks) {
    nh = min(static_cast<uint32_t>(hc >> 40), hub_cap);
    nchunks = static_cast<uint32_t>(hc & ((1ull << 40) - 1));
}

__device__ __forceinline__ uint32_t raise_threshold(uint32_t t, uint32_t delta) {
    return t >= kInf - delta ? kInf : t + delta;
}

// The far list that pushes go to after `tr` threshold raises.
__device__ __forceinline__ Sink far_sink(const Params &p, uint32_t tr) {
    return Sink{&p.ctrl->far_cnt[tr % 3], (tr & 1u) ? p.far1 : p.far0, p.far_cap, p.ctrl,
                &p.ctrl->far_min[tr % 3]};
}

// Next threshold: the far list's lower bound plus delta, so that every raise
// moves at least the closest listed vertex to the worklist.
__device__ __forceinline__ uint32_t next_threshold(uint32_t thresh, uint32_t far_min, uint32_t delta) {
    return raise_threshold(max(thresh, far_min), delta);
}


// ---------------------------------------------------------------------------
// BFS bottom-up invocation (direction optimization on a symmetric graph): a
// topology-driven ForAll over the vertices, where every unvisited vertex
// looks through its own neighbours for one in the current frontier and stops
// at the first hit.  Each vertex is decided by exactly one lane, so labels
// need no atomics; found vertices are pushed as usual so that a following
// top-down invocation has its worklist.
// ---------------------------------------------------------------------------

// Vertices per thread per step of the two full-vertex passes of a bottom-up
// invocation: their loads are issued together (measured on RMAT-22: BFS
// 0.543 ms against 0.583 ms with one vertex per step).
constexpr int kPullV = 4;

// Bitmaps for a bottom-up invocation at level `cur` that follows a top-down
// one: frontier = (level == cur), visited = (level != INF).  One ballot pair
// per 64 consecutive vertices; thread t of a step handles vertices
// base + j * blockDim.x + t, j < kPullV.  (After a bottom-up invocation the
// pull pass itself leaves both bitmaps current.)
__device__ __forceinline__ void build_pull_bitmaps(const Params &p, uint32_t cur, Team tm, uint32_t *frontier) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    const uint32_t step = blockDim.x * kPullV;
    const int lane = lane_id();
    for (uint32_t base = tm.id * step; base < n; base += tm.size * step) {
        uint32_t lv[kPullV];
#pragma unroll
        for (int j = 0; j < kPullV; ++j) {
            const uint32_t v = base + j * blockDim.x + threadIdx.x;
            lv[j] = v < n ? p.val[v] : kInf;
        }
#pragma unroll
        for (int j = 0; j < kPullV; ++j) {
            const uint32_t v = base + j * blockDim.x + threadIdx.x;
            const unsigned long long mv = __ballot(lv[j] != kInf);
            const unsigned long long mfr = __ballot(lv[j] == cur);
            const uint32_t v0 = v - static_cast<uint32_t>(lane);  // first vertex of this wavefront
            if (lane == 0 && v0 < n) {
                p.visited[v0 >> 5] = static_cast<uint32_t>(mv);
                frontier[v0 >> 5] = static_cast<uint32_t>(mfr);
            }
            if (lane == 32 && v < n) {
                p.visited[v >> 5] = static_cast<uint32_t>(mv >> 32);
                frontier[v >> 5] = static_cast<uint32_t>(mfr >> 32);
            }
        }
    }
}

// The pull pass: every unvisited vertex scans its neighbours kUMax at a time
// and stops at the first one in `frontier`.  The visited words and row
// offsets of a thread's kPullV vertices are loaded together first.  The
// vertices found form the next frontier: each wavefront writes their bits to
// `next_frontier` and adds them to `visited` (the 64 vertices of a ballot
// are consecutive and only their wavefront reads or writes those words in
// this pass), so a following bottom-up invocation needs no rebuild.
template <int B>
__device__ __forceinline__ void pull_level(const Params &p, uint32_t next, Team tm, Pushers &pu,
                                           unsigned long long &scanned, const uint32_t *frontier,
                                           uint32_t *next_frontier) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    constexpr uint32_t kStep = B * kPullV;
    for (uint32_t base = tm.id * kStep; base < n; base += tm.size * kStep) {
        uint32_t vw[kPullV];
        int rr0[kPullV], rr1[kPullV];
#pragma unroll
        for (int j = 0; j < kPullV; ++j) {
            const uint32_t v = base + j * B + threadIdx.x;
            vw[j] = v < n ? p.visited[v >> 5] : ~0u;
        }
#pragma unroll
        for (int j = 0; j < kPullV; ++j) {
            const uint32_t v = base + j * B + threadIdx.x;
            const bool unvisited = v < n && !((vw[j] >> (v & 31)) & 1u);
            rr0[j] = unvisited ? p.row_ptr[v] : 0;
            rr1[j] = unvisited ? p.row_ptr[v + 1] : 0;
        }
#pragma unroll
        for (int j = 0; j < kPullV; ++j) {
            const uint32_t v = base + j * B + threadIdx.x;
            const int r0 = rr0[j], r1 = rr1[j];
            int found = -1;
            for (int e0 = r0; e0 < r1; e0 += kUMax) {
                int u[kUMax];
                uint32_t fw[kUMax];
#pragma unroll
                for (int k = 0; k < kUMax; ++k) u[k] = e0 + k < r1 ? p.col[e0 + k] : -1;
#pragma unroll
                for (int k = 0; k < kUMax; ++k)
                    fw[k] = u[k] >= 0 ? frontier[static_cast<uint32_t>(u[k]) >> 5] : 0u;
#pragma unroll
                for (int k = 0; k < kUMax; ++k)
                    if (found < 0 && u[k] >= 0 && ((fw[k] >> (u[k] & 31)) & 1u)) found = u[k];
                scanned += static_cast<unsigned long long>(min(kUMax, r1 - e0));
                if (found >= 0) break;
            }
            if (found >= 0) {
                p.val[v] = next;
                if (p.parent) p.parent[v] = p.perm ? p.perm[found] : found;
                pu.mf += static_cast<unsigned long long>(r1 - r0);
            }
            const unsigned long long mf = __ballot(found >= 0);
            const int lane = lane_id();
            const uint32_t v0 = v - static_cast<uint32_t>(lane);  // first vertex of this wavefront
            if (lane == 0 && v0 < n) {
                next_frontier[v0 >> 5] = static_cast<uint32_t>(mf);
                p.visited[v0 >> 5] = vw[j] | static_cast<uint32_t>(mf);
            }
            if (lane == 32 && v < n) {
                next_frontier[v >> 5] = static_cast<uint32_t>(mf >> 32);
                p.visited[v >> 5] = vw[j] | static_cast<uint32_t>(mf >> 32);
            }
            pu.near(found >= 0, static_cast<int>(v));
        }
    }
}

// ---------------------------------------------------------------------------
// SSSP heavy pass as a pull (split symmetric graphs): every vertex u whose
// distance exceeds `lo` scans its heavy range for vertices listed in bucket
// `bucket` (their distances are final) and takes the smallest
// dist[v] + w(v, u) through the operator's relaxation, as if that one edge
// had been pushed.  Each u is decided by one lane.  `lo` is the smallest
// distance any vertex was expanded with in the bucket plus the step (a
// listed vertex's final distance is the one of its last expansion): a heavy
// edge (weight at least the step) from the bucket cannot bring any vertex to
// `lo` or below, so those vertices are skipped whatever the bucket's width.  (The threshold
// itself is no bound: it jumps over empty ranges, so a bucket can be wider
// than the step and vertices below it can still improve.)
// ---------------------------------------------------------------------------
// A vertex whose heavy range is longer than this is not scanned by one lane:
// it raises *big, and the caller runs the push pass after all.
constexpr int kPullMaxRange = 1024;

constexpr int kPullBatch = 8;

template <int B, class Op>
__device__ __forceinline__ void pull_heavy(const Params &p, const Op &hop, uint32_t lo, uint32_t bucket, Team tm,
                                           Pushers &pu, unsigned long long &scanned, uint32_t *big) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    bool saw_big = false;
    for (uint32_t base = tm.id * B; base < n; base += tm.size * B) {
        const uint32_t u = base + threadIdx.x;
        int e[Op::kU], d[Op::kU], sv[Op::kU];
        uint32_t dv[Op::kU];
        bool act[Op::kU], far[Op::kU];
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) {
            e[k] = 0;
            d[k] = 0;
            sv[k] = 0;
            dv[k] = 0;
            act[k] = false;
            far[k] = false;
        }
        if (u < n && p.val[u] > lo) {
            const uint32_t du = p.val[u];
            const int r0 = p.split[u];
            int r1 = p.row_ptr[u + 1];
            if (r1 - r0 > kPullMaxRange) {
                saw_big = true;
                r1 = r0;
            }
            unsigned long long best = du;
            // kPullBatch entries per step: their column loads, then their
            // bucket-stamp probes, are in flight together (a long range is
            // otherwise one dependent pair of loads per entry)
            for (int x0 = r0; x0 < r1; x0 += kPullBatch) {
                int vb[kPullBatch];
                uint32_t hb[kPullBatch];
#pragma unroll
                for (int k = 0; k < kPullBatch; ++k) vb[k] = x0 + k < r1 ? p.col[x0 + k] : -1;
#pragma unroll
                for (int k = 0; k < kPullBatch; ++k) hb[k] = vb[k] >= 0 ? p.hstamp[vb[k]] : ~bucket;
#pragma unroll
                for (int k = 0; k < kPullBatch; ++k) {
                    if (hb[k] != bucket) continue;
                    const int v = vb[k];
                    const uint32_t dvv = p.val[v];
                    const unsigned long long c =
                        static_cast<unsigned long long>(dvv) + static_cast<unsigned long long>(p.w[x0 + k]);
                    if (c < best) {
                        best = c;
                        e[0] = x0 + k;
                        sv[0] = v;
                        dv[0] = dvv;
                        act[0] = true;
                    }
                }
            }
            d[0] = static_cast<int>(u);
            scanned += static_cast<unsigned long long>(r1 - r0);
        }
        hop.relax(e, d, sv, dv, act, far, pu.fmin, pu.tries, pu.wins);
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) pu.near(act[k], d[k]);
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) pu.far(far[k], d[k]);
    }
    if (__syncthreads_or(saw_big) && threadIdx.x == 0) atomicOr(big, 1u);
}

// ---------------------------------------------------------------------------
// The outlined Iterate loop, run by one team (the whole grid of a
// single-query launch, or one group of a batched launch).  An invocation that
// deferred vertices to the grid tier has two team barriers (after phase A,
// after phase B); any other has one.  For SSSP an empty worklist with a
// non-empty far list is followed by a transfer invocation that raises the
// threshold by delta.  All control decisions read settled counters after a
// barrier, so they are uniform across the team.
// ---------------------------------------------------------------------------
struct LoopResult {
    uint32_t iterations;
    unsigned long long items;
    unsigned long long edges;   // CSR entries this workgroup scanned
    uint32_t max_frontier;
    unsigned long long fedges;  // out-degree sums of the worklists (this workgroup's share)
    uint32_t pulls;             // SSSP heavy passes run as a pull (uniform)
};

template <int B, class Op>
__device__ __forceinline__ LoopResult run_iterate(const Params &p, Smem<B> &sm, Team tm, BarrierState &bs) {
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    Ctrl *ctrl = p.ctrl;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, {}, {}, kInf};
    pu.hq.q = sm.queue_heavy[wid];
    // SSSP light/heavy split: expansions relax light ranges and list the
    // vertex for its bucket's heavy pass, which runs in the bucket's transfer
    // invocation (one barrier for both)
    const bool split = Op::kFar && p.split != nullptr;
    LoopResult r{0u, 0ull, 0ull, 0u, 0ull, 0u};
    // BFS direction choice (needs the frontier bitmap; symmetric graphs only)
    bool can_pull = !Op::kFar && p.frontier != nullptr;
    bool pull = false;
    bool bitmaps_current = false;  // the previous invocation was bottom-up: its bitmaps describe this one
    uint32_t *fr_cur = p.frontier, *fr_next = p.frontier2;
    unsigned long long m_seen = 0;  // out-degree sum of all worklists so far
    unsigned long long m_f = 0;     // out-degree sum of this invocation's worklist
    unsigned long long bu_seen = 0; // ctrl->bu_scan after the last bottom-up invocation
    if (can_pull) pu.deg_rp = p.row_ptr;
    const int32_t *in = p.wl0;
    int32_t *out = p.wl1;
    uint32_t it = 0;
    uint32_t tr = 0;                              // threshold raises so far
    uint32_t thresh = Op::kFar ? p.delta : kInf;  // near/far split point
    const bool lead = tm.id == 0 && tid == 0;
    // popped items when the bitmap was last refreshed: refresh again once the
    // newly reached vertices carry enough edges to repay a full scan
    unsigned long long refreshed = 0;
    unsigned long long hdone = 0;  // heavy edges of the buckets drained so far

    for (;; ++it) {
        uint32_t cnt_in = load_agent(&ctrl->cnt[it % 3]);
        if (cnt_in > p.cap) cnt_in = p.cap;  // overflowed pushes were dropped (error set)
        uint32_t far_n = 0, nheavy = 0;
        if (cnt_in == 0) {
            if (!Op::kFar) break;
            far_n = min(load_agent(&ctrl->far_cnt[tr % 3]), p.far_cap);
            if (split) nheavy = min(load_agent(&ctrl->hcnt[tr % 3]), p.hcap);
            if (far_n == 0 && nheavy == 0) break;
        }
        if (it >= p.max_iter) {
            if (lead) set_error(ctrl, kErrIterLimit, false);
            break;
        }
        r.items += cnt_in;
        r.max_frontier = max(r.max_frontier, cnt_in);
        if (lead) {
            store_agent(&ctrl->cnt[(it + 2) % 3], 0u);
            store_agent(&ctrl->tile[(it + 2) % 3], 0u);
            __hip_atomic_store(&ctrl->hub[(it + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctrl->mf[(it + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // read inside invocation it after a barrier of it: clear the next one's
            store_agent(&ctrl->hbig[(it + 1) % 3], 0u);
            if (cnt_in == 0) {
                store_agent(&ctrl->far_cnt[(tr + 2) % 3], 0u);
                store_agent(&ctrl->far_min[(tr + 2) % 3], kInf);
                store_agent(&ctrl->hcnt[(tr + 1) % 3], 0u);  // the next bucket's heavy list
                __hip_atomic_store(&ctrl->hsum[(tr + 1) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                store_agent(&ctrl->hmin[(tr + 1) % 3], kInf);
            }
            if (tracing(p, it)) trace_start(p, it, cnt_in);
        }
        pu.sk = Sink{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl};
        unsigned long long *hub_ctr = &ctrl->hub[it % 3];
        if (cnt_in == 0) {
            // transfer invocation (SSSP only): far list tr -> next worklist / far list tr + 1.
            // With an empty far list (only a heavy pass left) the threshold
            // rises by one step, so the heavy results keep their bucket order.
            // heavy entries listed by the drained bucket, and by all before it
            const unsigned long long hs =
                p.pull_heavy_div ? __hip_atomic_load(&ctrl->hsum[tr % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : 0ull;
            const unsigned long long open = p.heavy_m > hdone ? p.heavy_m - hdone : 0ull;
            hdone += hs;
            // once nearly every heavy entry has been listed, the buckets left
            // hold few vertices: wider ones cost fewer invocations
            const uint32_t step = (p.step_grow && p.heavy_m && hdone * 8 >= p.heavy_m * 7 &&
                                   p.delta <= kInf / p.step_grow)
                                      ? p.delta * p.step_grow
                                      : p.delta;
            uint32_t t_new =
                far_n ? next_threshold(thresh, load_agent(&ctrl->far_min[tr % 3]), step)
                      : raise_threshold(thresh, step);
            // the last buckets of a scale-free graph hold few vertices each,
            // and each costs invocations (barriers): once the far list is
            // small next to the work done, finish without a threshold
            if (p.tail_div && far_n &&
                static_cast<unsigned long long>(far_n) * p.tail_div < r.items)
                t_new = kInf;
            if (p.visited && r.items - refreshed >= p.t_bitmap) {
                refresh_bitmap(p, tm, thresh);  // every distance below thresh is final
                refreshed = r.items;
            }
            pu.skf = far_sink(p, tr + 1);
            pu.skh = Sink{};
            pu.hsum_out = nullptr;
            far_transfer<B>((tr & 1u) ? p.far1 : p.far0, far_n, static_cast<uint32_t>(p.n), thresh, t_new,
                            p.val, p.far_flag, p.stamp, it, pu, tm);
            // heavy pass of the drained bucket (split graphs): its vertices'
            // distances are final, so each heavy edge is relaxed once; the
            // results (at least thresh) go to the next worklist (below t_new)
            // or the far list.  Push: the listed vertices' heavy ranges.
            // Pull, when those ranges are many: each unsettled vertex scans
            // its own heavy range for the bucket's vertices (the same edges
            // seen from the other end of a symmetric graph).
            const unsigned long long edges_before = r.edges;
            const Op hop = make_op<Op>(p, it, t_new, tr, true);
            // Pull only for a bucket no wider than the step (the smallest
            // expanded distance plus the step reaches the drained threshold):
            // then the vertices it scans are those beyond the threshold.
            const uint32_t hm = load_agent(&ctrl->hmin[tr % 3]);
            const uint32_t lo = hm >= kInf - p.delta ? kInf : hm + p.delta;
            bool pull_h = nheavy > 0 && p.pull_heavy_div && lo >= thresh &&
                          hs * p.pull_heavy_div >= static_cast<unsigned long long>(p.n) &&
                          (p.pull_open_div == 0 || hs * p.pull_open_div >= open);
            bool pulled = false;
            if (pull_h) {
                if constexpr (Op::kFar) pull_heavy<B, Op>(p, hop, lo, tr, tm, pu, r.edges, &ctrl->hbig[it % 3]);
                drain_all<B, Op>(pu, sm);
                if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
                // an unsettled vertex with a long heavy range was left out: the
                // push pass relaxes every listed vertex's heavy edges after all
                // (the pull's relaxations were real edges: nothing to undo)
                pulled = load_agent(&ctrl->hbig[it % 3]) == 0u;
                r.pulls += pulled ? 1u : 0u;
            }
            if (!pulled) {
                if (nheavy > 0)
                    expand<B, Op>(p.hlist, nheavy, static_cast<uint32_t>(p.n), p.row_ptr, p.col, hop, sm, pu,
                                  p.t_wave, p.t_block, p.t_grid, p.hub_v, p.hub_base, p.hub_cap, hub_ctr, r.edges, tm,
                                  &ctrl->tile[it % 3]);
                drain_all<B, Op>(pu, sm);
                if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
                if (nheavy > 0 && p.t_grid > 0) {
                    uint32_t nh, nchunks;
                    hub_counts(__hip_atomic_load(hub_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), p.hub_cap,
                               nh, nchunks);
                    if (nh > 0) {
                        expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, hop, sm, pu, tm);
                        drain_all<B, Op>(pu, sm);
                        if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
                    }
                }
            }
            if ((nheavy > 0 || pulled) && tracing(p, it)) trace_level(p, it, r.edges - edges_before, hub_ctr, tm, pu);
            thresh = t_new;
            ++tr;
        } else if (can_pull && ([&] {
                       // uniform: the settled out-degree sum of this worklist
                       m_f = __hip_atomic_load(&ctrl->mf[it % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                       m_seen += m_f;
                       const long long m_u = p.m - static_cast<long long>(m_seen);
                       if (!pull) pull = static_cast<long long>(m_f) * p.do_alpha > m_u;
                       else pull = static_cast<unsigned long long>(cnt_in) * p.do_beta >=
                                   static_cast<unsigned long long>(p.n);
                       if (pull && tid == 0 && tm.id == 0) r.fedges += m_f;
                       return pull;
                   }())) {
            // bottom-up invocation: bitmaps, barrier, pull
            pu.mf_out = &ctrl->mf[(it + 1) % 3];
            if (!bitmaps_current) {
                build_pull_bitmaps(p, it, tm, fr_cur);
                if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
            }
            const unsigned long long edges_before = r.edges;
            pull_level<B>(p, it + 1, tm, pu, r.edges, fr_cur, fr_next);
            uint32_t *const fr_t = fr_cur;
            fr_cur = fr_next;
            fr_next = fr_t;
            bitmaps_current = true;
            refreshed = r.items;  // the visited bitmap is exact again
            drain_all<B, Op>(pu, sm);
            add_block_total<B>(r.edges - edges_before, &ctrl->bu_scan);
            if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
            // uniform: a bottom-up invocation that scanned more than twice the
            // edges the top-down one would have (a high-diameter graph, where
            // unvisited vertices rarely touch the frontier) ends bottom-up for
            // the query
            const unsigned long long bu_now =
                __hip_atomic_load(&ctrl->bu_scan, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (bu_now - bu_seen > 2 * m_f) {
                can_pull = false;
                pull = false;
            }
            bu_seen = bu_now;
            if (tracing(p, it)) trace_level(p, it, r.edges - edges_before, hub_ctr, tm, pu);
        } else {
            bitmaps_current = false;  // top-down labels are not in the bitmaps
            pu.skf = far_sink(p, tr);
            pu.skh = split ? Sink{&ctrl->hcnt[tr % 3], p.hlist, p.hcap, ctrl, nullptr} : Sink{};
            pu.hsum_out = (split && p.pull_heavy_div) ? &ctrl->hsum[tr % 3] : nullptr;
            pu.hmin_out = &ctrl->hmin[tr % 3];
            pu.mf_out = &ctrl->mf[(it + 1) % 3];
            const unsigned long long edges_before = r.edges;
            if (!Op::kFar && p.visited && r.items - refreshed >= p.t_bitmap) {
                refresh_bitmap(p, tm, kInf);  // BFS: visited = labelled
                refreshed = r.items;
            }
            const Op op = make_op<Op>(p, it, thresh, tr, false);
            const bool tr_on = tracing(p, it);
            unsigned long long busy_a = tr_on ? wall_clock64() : 0ull, busy_b = 0;
            expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, pu, p.t_wave,
                          p.t_block, p.t_grid, p.hub_v, p.hub_base, p.hub_cap, hub_ctr, r.edges, tm,
                          &ctrl->tile[it % 3]);
            drain_all<B, Op>(pu, sm);
            if (tr_on) busy_a = wall_clock64() - busy_a;
            if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
            if (p.t_grid > 0) {
                uint32_t nh, nchunks;
                hub_counts(__hip_atomic_load(hub_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), p.hub_cap,
                           nh, nchunks);
                if (nh > 0) {
                    if (tr_on) busy_b = wall_clock64();
                    if (lead && tr_on) p.trace[kTraceWords * it + 4] = busy_b;
                    expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, op, sm, pu, tm);
                    drain_all<B, Op>(pu, sm);
                    if (tr_on) busy_b = wall_clock64() - busy_b;
                    if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag, tm)) break;
                }
            }
            r.fedges += r.edges - edges_before;
            if (tr_on) trace_level(p, it, r.edges - edges_before, hub_ctr, tm, pu, busy_a, busy_b);
        }
        const int32_t *t = in;
        in = out;
        out = const_cast<int32_t *>(t);
    }
    r.iterations = it;
    return r;
}

// Statistics and completion of a query run by a team: the last workgroup of
// the team to finish publishes the caller's stats block.
template <int B>
__device__ __forceinline__ void finish_query(const Params &p, const LoopResult &r, Team tm) {
    Ctrl *ctrl = p.ctrl;
    add_block_total<B>(r.edges, &ctrl->edges);
    add_block_total<B>(r.fedges, &ctrl->fedges);
    if (threadIdx.x == 0) {
        if (tm.id == 0) {
            if (kTraceWords * r.iterations < p.trace_len) p.trace[kTraceWords * r.iterations] = wall_clock64();
            ctrl->iterations = r.iterations;
            ctrl->items = r.items;
            ctrl->max_frontier = r.max_frontier;
            ctrl->pulls = r.pulls;
            ctrl->grid = static_cast<int32_t>(tm.size);
            ctrl->block = B;
        }
        const uint32_t prev = __hip_atomic_fetch_add(&ctrl->done, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev == tm.size - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            publish_stats(p);
        }
    }
}

// Results of a relabelled graph under caller ids: a gather over caller ids
// (coalesced reads of inv and coalesced writes, one random read of the
// internal-id values each), by the whole team after its last barrier.
__device__ __forceinline__ void map_to_caller(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t o = tm.id * blockDim.x + threadIdx.x; o < n; o += tm.size * blockDim.x) {
        const int32_t v = p.inv[o];
        p.out_caller[o] = p.val[v];
        if (p.parent_caller) p.parent_caller[o] = p.parent[v];
    }
}

// One query per cooperative launch: the whole grid is the team.
template <int B, class Op>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(fit_waves<B, Op::kMinWaves>()))) void persistent_kernel(
    Params p) {
    __shared__ Smem<B> sm;
    const Team tm = whole_grid();
    BarrierState bs = make_barrier_state(p.wd_ticks, p.barrier);
    const LoopResult r = run_iterate<B, Op>(p, sm, tm, bs);
    // every value is final: the loop ended after a barrier that followed the
    // last write of any workgroup
    if (p.inv) map_to_caller(p, tm);
    finish_query<B>(p, r, tm);
}

// ---------------------------------------------------------------------------
// Un-outlined form: invocation `p.it` is one launch of level_kernel (phase
// A) and one of hub_level_kernel (phase B, returns at once when nothing was
// deferred), or one launch of transfer_kernel for an SSSP threshold raise;
// the host reads the counters back after each invocation and decides what to
// launch next.  The host keeps the threshold (p.thresh) and the number of
// raises (p.far_tr).
// ---------------------------------------------------------------------------
template <int B, class Op>
__global__ __launch_bounds__(B) void level_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    Ctrl *ctrl = p.ctrl;
    const uint32_t it = p.it;
    unsigned long long edges = 0;
    const int32_t *in = (it & 1u) ? p.wl1 : p.wl0;
    int32_t *out = (it & 1u) ? p.wl0 : p.wl1;
    uint32_t cnt_in = ctrl->cnt[it % 3];
    if (cnt_in > p.cap) cnt_in = p.cap;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl, nullptr},
               far_sink(p, p.far_tr), kInf};
    if (blockIdx.x == 0 && tid == 0 && tracing(p, it)) trace_start(p, it, cnt_in);
    if (p.refresh && p.visited) refresh_bitmap(p, whole_grid(), kInf);
    const Op op = make_op<Op>(p, it, p.thresh);
    expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, pu, p.t_wave, p.t_block,
                  p.t_grid, p.hub_v, p.hub_base, p.hub_cap, &ctrl->hub[it % 3], edges, whole_grid(),
                  &ctrl->tile[it % 3]);
    drain_all<B, Op>(pu, sm);
    add_block_total<B>(edges, &ctrl->edges);
    add_block_total<B>(edges, &ctrl->fedges);  // top-down only: every worklist edge is scanned
    if (tid == 0 && blockIdx.x == 0) {
        ctrl->cnt[(it + 2) % 3] = 0;
        ctrl->tile[(it + 2) % 3] = 0;
        ctrl->hub[(it + 2) % 3] = 0;
        ctrl->iterations = it + 1;
        ctrl->items += cnt_in;
        ctrl->max_frontier = max(ctrl->max_frontier, cnt_in);
        ctrl->grid = static_cast<int32_t>(gridDim.x);
        ctrl->block = B;
    }
}

template <int B, class Op>
__global__ __launch_bounds__(B) void hub_level_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int wid = threadIdx.x / kWave;
    Ctrl *ctrl = p.ctrl;
    const uint32_t it = p.it;
    uint32_t nh, nchunks;
    hub_counts(ctrl->hub[it % 3], p.hub_cap, nh, nchunks);
    if (nh == 0) return;  // uniform across the grid
    int32_t *out = (it & 1u) ? p.wl0 : p.wl1;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl, nullptr},
               far_sink(p, p.far_tr), kInf};
    const Op op = make_op<Op>(p, it, p.thresh);
    expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, op, sm, pu, whole_grid());
    drain_all<B, Op>(pu, sm);
}

// SSSP threshold raise of the un-outlined form: far list p.far_tr ->
// next worklist / far list p.far_tr + 1, threshold p.thresh -> p.t_new.
template <int B>
__global__ __launch_bounds__(B) void transfer_kernel(Params p, uint32_t far_n, uint32_t t_new) {
    __shared__ Smem<B> sm;
    const int wid = threadIdx.x / kWave;
    Ctrl *ctrl = p.ctrl;
    const uint32_t it = p.it;
    const uint32_t tr = p.far_tr;
    int32_t *out = (it & 1u) ? p.wl0 : p.wl1;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl, nullptr},
               far_sink(p, tr + 1), kInf};
    if (blockIdx.x == 0 && threadIdx.x == 0 && tracing(p, it)) {
        trace_start(p, it, 0u);
    }
    if (p.refresh && p.visited) refresh_bitmap(p, whole_grid(), p.thresh);
    far_transfer<B>((tr & 1u) ? p.far1 : p.far0, far_n, static_cast<uint32_t>(p.n), p.thresh, t_new, p.val,
                    p.far_flag, p.stamp, it, pu, whole_grid());
    drain_all<B, SsspOp>(pu, sm);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->cnt[(it + 2) % 3] = 0;
        ctrl->tile[(it + 2) % 3] = 0;
        ctrl->hub[(it + 2) % 3] = 0;
        ctrl->far_cnt[(tr + 2) % 3] = 0;
        ctrl->far_min[(tr + 2) % 3] = kInf;
        ctrl->iterations = it + 1;
    }
}

// Host-loop epilogue and the iteration-limit check of the un-outlined form.
__global__ void finish_kernel(Params p, int hit_limit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t it = p.ctrl->iterations;
        if (kTraceWords * it < p.trace_len) p.trace[kTraceWords * it] = wall_clock64();
        if (hit_limit) set_error(p.ctrl, kErrIterLimit, false);
        publish_stats(p);
    }
}

// SSSP parent pass over the identity worklist of all n vertices (the grid
// tier is off: ranges of every size are expanded in place).
template <int B>
__global__ __launch_bounds__(B) void sssp_parent_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int wid = threadIdx.x / kWave;
    Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{nullptr, nullptr, 0u, p.ctrl, nullptr},
               Sink{nullptr, nullptr, 0u, p.ctrl, nullptr}, kInf};
    unsigned long long edges = 0;
    const SsspParentOp op{p.val, p.w, p.parent, p.src, p.perm};
    expand<B, SsspParentOp>(nullptr, static_cast<uint32_t>(p.n), static_cast<uint32_t>(p.n), p.row_ptr, p.col,
                            op, sm, pu, p.t_wave, p.t_block, 0, nullptr, nullptr, 0u, nullptr, edges,
                            whole_grid(), nullptr);
}

// Relabelled graph: results computed under internal ids (vals, parents
// already caller ids) go to the caller's arrays under caller ids.
__global__ void scatter_results_kernel(int32_t n, const int32_t *perm, const uint32_t *val, const int32_t *par,
                                       uint32_t *out, int32_t *out_parent) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t o = perm[v];
        out[o] = val[v];
        if (out_parent) out_parent[o] = par[v];
    }
}

// On-device CSR validation: row_ptr[0] == 0, monotone, row_ptr[n] == m,
// col in [0, n), w >= 1.  Sets *bad to 1 on any violation; also sums the
// weights and takes the largest out-degree (one atomic per wavefront).
__global__ void validate_kernel(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                                const uint32_t *w, uint32_t *bad, unsigned long long *wsum, uint32_t *maxdeg) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (tid == 0 && (row_ptr[0] != 0 || static_cast<int64_t>(row_ptr[n]) != m)) atomicOr(bad, 1u);
    int32_t dmax = 0;
    for (uint32_t v = tid; v < static_cast<uint32_t>(n); v += stride) {
        const int32_t d = row_ptr[v + 1] - row_ptr[v];
        if (d < 0) atomicOr(bad, 1u);
        dmax = d > dmax ? d : dmax;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int32_t x = __shfl_xor(dmax, o);
        dmax = x > dmax ? x : dmax;
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && dmax > 0) atomicMax(maxdeg, static_cast<uint32_t>(dmax));
    unsigned long long ws = 0;
    for (uint64_t e = tid; e < static_cast<uint64_t>(m); e += stride) {
        const int32_t d = col[e];
        if (d < 0 || d >= n) atomicOr(bad, 1u);
        if (w) {
            if (w[e] == 0u) atomicOr(bad, 1u);
            ws += w[e];
        }
    }
    if (w && ws) atomicAdd(wsum, ws);
}

}  // namespace irgl
