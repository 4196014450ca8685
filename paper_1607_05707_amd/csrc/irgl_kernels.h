// gfx950 kernels of the data-driven BFS/SSSP hot path.
//
//   * Frontier expansion: the outer ForAll over the incoming worklist
//     (Section 3.1: consecutive items on consecutive lanes) with nested edge
//     parallelism for the inner ForAll over graph.edges(n) (Sections 4.1 and
//     4.3).  Four tiers by out-degree: grid (all workgroups split the edge
//     ranges of the largest vertices into equal chunks after a grid barrier),
//     workgroup, wavefront, and a prefix-sum gather that deals the small
//     ranges of a workgroup to consecutive lanes.  Every tier hands each lane
//     U edges per round so that U independent memory chains are in flight.
//   * Relax operators, written as phases over a lane's U edges (all loads of
//     one phase are issued before any result is used): the BFS
//     check-and-label of the Section 4.1 listing made exactly-once with a
//     compare-and-swap, behind a visited-bitmap filter; the SSSP "distance
//     improved" test with atomicMin and a per-invocation push stamp.
//   * The outlined Iterate loop (Sections 4.2 and 4.3): one persistent,
//     co-resident grid runs every invocation, separated by the grid barrier,
//     swapping the in/out worklists each time.
//   * The un-outlined form: one launch per invocation.
//   * Initialisation (the worklist initializer [src]) and the SSSP parent pass.
#pragma once

#include "irgl_device.h"

namespace irgl {

constexpr int kQueueCap = 256;  // LDS staging entries per wavefront
constexpr int kU = 4;           // edges per lane per round (memory-level parallelism)

// Shared-memory layout of the frontier kernels for workgroup size B.
template <int B>
struct Smem {
    static constexpr int NW = B / kWave;
    int gather_edge[B * kU];       // edge index of each slot of the current gather window
    uint16_t gather_owner[B * kU]; // thread whose vertex owns that edge
    int vtx[B];                    // popped vertex of each thread
    uint32_t vval[B];              // its per-vertex value (SSSP distance at pop)
    int wsum[NW];                  // per-wavefront degree sums for the workgroup scan
    int fill[NW];                  // per-wavefront queue fill at the workgroup drain
    int queue[NW][kQueueCap];
    int owner;                     // workgroup-tier vertex owner
    int big_r0, big_r1, big_v;
    uint32_t big_val;
    uint32_t base;
    int flag;
    int hub_h;                     // grid tier: first deferred vertex of this workgroup
};

struct Params {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    uint32_t *val;        // level (BFS) or dist (SSSP)
    int32_t *parent;      // optional
    uint32_t *stamp;      // SSSP push stamps
    int32_t *wl0;
    int32_t *wl1;
    int32_t *hub_v;       // grid tier: deferred vertices of the current invocation
    uint32_t *hub_base;   // grid tier: first chunk of each deferred vertex
    uint32_t hub_cap;
    Ctrl *ctrl;
    Stats *dstats;        // optional
    uint32_t cap;         // worklist capacity
    uint32_t max_iter;
    int32_t t_wave;
    int32_t t_block;
    int32_t t_grid;       // 0 disables the grid tier
    int32_t src;
    uint32_t it;          // host-loop mode: the invocation to run
    unsigned long long wd_ticks;
    const volatile int32_t *abort_flag;
    uint32_t *visited;    // BFS visited bitmap, ceil(n / 32) words
    uint32_t t_bitmap;    // refresh the bitmap when the incoming worklist is this large
    uint32_t trace_len;
    unsigned long long *trace;
};

// ---------------------------------------------------------------------------
// Relax operators.  relax(e, d, sv, sval, act) receives U scanned edges
// e[k] = (sv[k] -> d[k]) of this lane, act[k] marking the live ones, and
// leaves act[k] true for each destination that must be pushed.
// ---------------------------------------------------------------------------
struct BfsOp {
    static constexpr bool kPush = true;
    uint32_t *level;
    int32_t *parent;
    const uint32_t *visited;  // bitmap: a set bit means "visited" (never a false positive)
    uint32_t next;            // label of vertices found in this invocation
    __device__ __forceinline__ uint32_t vertex_value(int) const { return 0u; }
    __device__ __forceinline__ bool active(uint32_t) const { return true; }
    __device__ __forceinline__ void relax(const int (&)[kU], const int (&d)[kU], const int (&sv)[kU],
                                          const uint32_t (&)[kU], bool (&act)[kU]) const {
        // Cheapest filter first: the n/8-byte bitmap stays resident in L2.
        // (visited is null when the bitmap is disabled: a uniform branch)
        if (visited) {
            uint32_t wd[kU];
#pragma unroll
            for (int k = 0; k < kU; ++k) wd[k] = act[k] ? visited[static_cast<uint32_t>(d[k]) >> 5] : 0u;
#pragma unroll
            for (int k = 0; k < kU; ++k) act[k] = act[k] && !(wd[k] & (1u << (d[k] & 31)));
        }
        // A plain (possibly stale) load of the level filters most of the rest;
        // stale values can only read INF, and the CAS decides.
        uint32_t lv[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) lv[k] = act[k] ? level[d[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            act[k] = act[k] && lv[k] == kInf;
            if (act[k]) act[k] = atomicCAS(&level[d[k]], kInf, next) == kInf;
        }
        if (parent) {
#pragma unroll
            for (int k = 0; k < kU; ++k)
                if (act[k]) parent[d[k]] = sv[k];
        }
    }
};

struct SsspOp {
    static constexpr bool kPush = true;
    uint32_t *dist;
    const uint32_t *w;
    uint32_t *stamp;
    uint32_t it;
    Ctrl *ctrl;
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return dist[v]; }
    __device__ __forceinline__ bool active(uint32_t) const { return true; }
    __device__ __forceinline__ void relax(const int (&e)[kU], const int (&d)[kU], const int (&)[kU],
                                          const uint32_t (&dv)[kU], bool (&act)[kU]) const {
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
            act[k] = act[k] && nd[k] < cur[k];
            if (act[k]) act[k] = nd[k] < atomicMin(&dist[d[k]], nd[k]);
        }
        // push d at most once per invocation
#pragma unroll
        for (int k = 0; k < kU; ++k) cur[k] = act[k] ? stamp[d[k]] : it;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            act[k] = act[k] && cur[k] != it;
            if (act[k]) act[k] = atomicExch(&stamp[d[k]], it) != it;
        }
    }
};

// Deterministic SSSP parents after convergence: the smallest-id tight
// predecessor of every reached vertex (unsigned min over -1 = 0xFFFFFFFF).
struct SsspParentOp {
    static constexpr bool kPush = false;
    const uint32_t *dist;
    const uint32_t *w;
    int32_t *parent;
    int32_t src;
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return dist[v]; }
    __device__ __forceinline__ bool active(uint32_t dv) const { return dv != kInf; }
    __device__ __forceinline__ void relax(const int (&e)[kU], const int (&d)[kU], const int (&sv)[kU],
                                          const uint32_t (&dv)[kU], bool (&act)[kU]) const {
        uint32_t s[kU], cur[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) s[k] = act[k] ? dv[k] + w[e[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) cur[k] = act[k] ? dist[d[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            if (act[k] && d[k] != src && s[k] == cur[k] && s[k] >= dv[k])
                atomicMin(reinterpret_cast<uint32_t *>(&parent[d[k]]), static_cast<uint32_t>(sv[k]));
            act[k] = false;
        }
    }
};

// Where one invocation's pushes go.
struct Sink {
    uint32_t *cnt_out;
    int32_t *out;
    uint32_t cap;
    Ctrl *ctrl;
};

// Relax U edges of one lane and push the survivors (all 64 lanes call it).
template <class Op>
__device__ __forceinline__ void relax_and_push(const Op &op, const int32_t *__restrict__ col,
                                               const int (&e)[kU], bool (&act)[kU], const int (&sv)[kU],
                                               const uint32_t (&sval)[kU], WaveQueue<kQueueCap> &wq,
                                               const Sink &sk) {
    int d[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) d[k] = act[k] ? col[e[k]] : 0;
    op.relax(e, d, sv, sval, act);
    if (Op::kPush) {
#pragma unroll
        for (int k = 0; k < kU; ++k) wq.push(act[k], d[k], sk.cnt_out, sk.out, sk.cap, sk.ctrl);
    }
}

// A group of `width` lanes (lane index `li` in it) strides the range
// [r0, r1) of vertex sv, U edges per lane per round.  The trip count is
// uniform across the group.
template <class Op>
__device__ __forceinline__ void stride_range(const Op &op, const int32_t *__restrict__ col, int r0,
                                             int r1, int sv, uint32_t sval, int li, int width,
                                             WaveQueue<kQueueCap> &wq, const Sink &sk) {
    int svs[kU];
    uint32_t svals[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
        svs[k] = sv;
        svals[k] = sval;
    }
    for (int e0 = r0; e0 < r1; e0 += width * kU) {
        int e[kU];
        bool act[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            e[k] = e0 + k * width + li;
            act[k] = e[k] < r1;
        }
        relax_and_push(op, col, e, act, svs, svals, wq, sk);
    }
}

// ---------------------------------------------------------------------------
// Phase A of one invocation: nested-parallel expansion of the incoming
// worklist.  `in == nullptr` means the identity worklist 0..cnt_in-1.
// Vertices of out-degree >= t_grid (t_grid > 0) are appended to the
// grid-tier list (hub_v / hub_base, counted by *hub_ctr) instead of being
// expanded here.  Every thread of every workgroup must call it (it
// synchronises the workgroup).
// ---------------------------------------------------------------------------
template <int B, class Op>
__device__ __forceinline__ void expand(const int32_t *__restrict__ in, uint32_t cnt_in, uint32_t n,
                                       const int32_t *__restrict__ row_ptr,
                                       const int32_t *__restrict__ col, const Op &op, Smem<B> &sm,
                                       WaveQueue<kQueueCap> &wq, const Sink &sk, int t_wave,
                                       int t_block, int t_grid, int32_t *hub_v, uint32_t *hub_base,
                                       uint32_t hub_cap, unsigned long long *hub_ctr,
                                       unsigned long long &edges) {
    constexpr int NW = B / kWave;
    constexpr int kChunk = B * kU;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wid = tid / kWave;
    const uint32_t stride = gridDim.x * B;

    for (uint32_t base = blockIdx.x * B; base < cnt_in; base += stride) {
        const uint32_t i = base + tid;
        int v = -1, r0 = 0, r1 = 0;
        uint32_t val = 0;
        if (i < cnt_in) {
            v = in ? in[i] : static_cast<int>(i);
            if (static_cast<uint32_t>(v) >= n) {  // never expected: a corrupt worklist entry
                set_error(sk.ctrl, kErrInternal, false);
                v = -1;
            } else {
                val = op.vertex_value(v);
                if (op.active(val)) {
                    r0 = row_ptr[v];
                    r1 = row_ptr[v + 1];
                }
            }
        }
        int deg = r1 - r0;
        edges += static_cast<unsigned long long>(deg);

        // Tier 0: defer the largest ranges to the grid-wide phase.
        if (t_grid > 0 && deg >= t_grid) {
            const unsigned long long chunks =
                (static_cast<unsigned long long>(deg) + kChunk - 1) / kChunk;
            const unsigned long long old = atomicAdd(hub_ctr, (1ull << 40) | chunks);
            const uint32_t slot = static_cast<uint32_t>(old >> 40);
            if (slot < hub_cap) {
                hub_v[slot] = v;
                hub_base[slot] = static_cast<uint32_t>(old & ((1ull << 40) - 1));
                deg = 0;
            }  // else: list full; the vertex is expanded here (cannot happen: cap >= m / t_grid + 1)
        }

        // Tier 1: the whole workgroup strides one large neighbour range at a time.
        while (__syncthreads_or(deg >= t_block)) {
            if (deg >= t_block) sm.owner = tid;
            __syncthreads();
            if (sm.owner == tid) {
                sm.big_r0 = r0;
                sm.big_r1 = r1;
                sm.big_v = v;
                sm.big_val = val;
                deg = 0;
            }
            __syncthreads();
            stride_range(op, col, sm.big_r0, sm.big_r1, sm.big_v, sm.big_val, tid, B, wq, sk);
        }

        // Tier 2: one wavefront strides one medium neighbour range at a time.
        for (;;) {
            const unsigned long long m = __ballot(deg >= t_wave);
            if (m == 0ull) break;
            const int leader = __ffsll(static_cast<long long>(m)) - 1;
            const int w0 = __shfl(r0, leader, kWave);
            const int w1 = __shfl(r1, leader, kWave);
            const int wv = __shfl(v, leader, kWave);
            const uint32_t wval = __shfl(val, leader, kWave);
            if (lane == leader) deg = 0;
            stride_range(op, col, w0, w1, wv, wval, lane, kWave, wq, sk);
        }

        // Tier 3: concatenate the remaining small ranges of the workgroup with
        // an exclusive prefix sum and deal edges to consecutive lanes.
        const int incl = wave_inclusive_scan(deg);
        if (lane == kWave - 1) sm.wsum[wid] = incl;
        sm.vtx[tid] = v;
        sm.vval[tid] = val;
        __syncthreads();
        int total = 0, wpre = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int s = sm.wsum[k];
            wpre += (k < wid) ? s : 0;
            total += s;
        }
        const int excl = wpre + incl - deg;
        for (int done = 0; done < total; done += kChunk) {
            const int lo = max(excl, done);
            const int hi = min(excl + deg, done + kChunk);
            for (int k = lo; k < hi; ++k) {
                sm.gather_edge[k - done] = r0 + (k - excl);
                sm.gather_owner[k - done] = static_cast<uint16_t>(tid);
            }
            __syncthreads();
            int e[kU], sv[kU];
            uint32_t sval[kU];
            bool act[kU];
#pragma unroll
            for (int k = 0; k < kU; ++k) {
                const int slot = k * B + tid;
                act[k] = slot < total - done;
                const int o = act[k] ? sm.gather_owner[slot] : 0;
                e[k] = act[k] ? sm.gather_edge[slot] : 0;
                sv[k] = sm.vtx[o];
                sval[k] = sm.vval[o];
            }
            relax_and_push(op, col, e, act, sv, sval, wq, sk);
            __syncthreads();
        }
    }
}

// Phase B (grid tier): every workgroup takes an equal contiguous share of
// the chunks of the deferred vertices (a chunk is B*U edges of one vertex;
// hub_base[] is ascending because slots and chunk bases come from one
// packed counter).  Called by all threads of every workgroup.
template <int B, class Op>
__device__ __forceinline__ void expand_hubs(uint32_t nhubs, uint32_t nchunks, const int32_t *hub_v,
                                            const uint32_t *hub_base,
                                            const int32_t *__restrict__ row_ptr,
                                            const int32_t *__restrict__ col, const Op &op, Smem<B> &sm,
                                            WaveQueue<kQueueCap> &wq, const Sink &sk) {
    constexpr int kChunk = B * kU;
    const unsigned long long G = gridDim.x;
    const uint32_t lo = static_cast<uint32_t>(nchunks * static_cast<unsigned long long>(blockIdx.x) / G);
    const uint32_t hi = static_cast<uint32_t>(nchunks * static_cast<unsigned long long>(blockIdx.x + 1) / G);
    if (lo >= hi) return;  // uniform across the workgroup
    if (threadIdx.x == 0) {
        // the last deferred vertex whose first chunk is <= lo
        uint32_t a = 0, b = nhubs;
        while (b - a > 1) {
            const uint32_t mid = (a + b) / 2;
            if (hub_base[mid] <= lo) a = mid;
            else b = mid;
        }
        sm.hub_h = static_cast<int>(a);
    }
    __syncthreads();
    uint32_t h = static_cast<uint32_t>(sm.hub_h);
    uint32_t c = lo;
    while (c < hi && h < nhubs) {
        const int v = hub_v[h];
        const uint32_t cb = hub_base[h];
        const int r0 = row_ptr[v], r1 = row_ptr[v + 1];
        const uint32_t nch = static_cast<uint32_t>((r1 - r0 + kChunk - 1) / kChunk);
        const uint32_t c_end = min(hi, cb + nch);
        const int e_lo = r0 + static_cast<int>((c - cb) * kChunk);
        const int e_hi = min(r1, r0 + static_cast<int>((c_end - cb) * kChunk));
        const uint32_t val = op.vertex_value(v);
        stride_range(op, col, e_lo, e_hi, v, val, threadIdx.x, B, wq, sk);
        c = c_end;
        ++h;
    }
}

// ---------------------------------------------------------------------------
// Initialisation: val = INF except val[src] = 0; parent = -1 except
// parent[src] = src; stamps = INF; bitmap = {src}; in = [src]; counters and
// stats cleared.
// ---------------------------------------------------------------------------
__global__ void init_kernel(Params p, int with_stamp) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool s = static_cast<int>(i) == p.src;
        p.val[i] = s ? 0u : kInf;
        if (p.parent) p.parent[i] = s ? p.src : -1;
        if (with_stamp) p.stamp[i] = kInf;
        if (p.visited && (i & 31u) == 0u)
            p.visited[i >> 5] = (static_cast<uint32_t>(p.src) >> 5 == i >> 5)
                                    ? (1u << (p.src & 31)) : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl *c = p.ctrl;
        c->cnt[0] = 1;
        c->cnt[1] = 0;
        c->cnt[2] = 0;
        for (int k = 0; k < 3; ++k) c->hub[k] = 0;
        c->bar_gen = 0;
        c->bar_top = 0;
        for (int g = 0; g < kBarGroups; ++g) c->bar_grp[g].count = 0;
        c->error = 0;
        c->fatal = 0;
        c->done = 0;
        c->iterations = 0;
        c->max_frontier = 0;
        c->items = 0;
        c->edges = 0;
        p.wl0[0] = p.src;
    }
}

template <class Op>
__device__ __forceinline__ Op make_op(const Params &p, uint32_t it);

template <>
__device__ __forceinline__ SsspOp make_op<SsspOp>(const Params &p, uint32_t it) {
    return SsspOp{p.val, p.w, p.stamp, it, p.ctrl};
}

template <>
__device__ __forceinline__ BfsOp make_op<BfsOp>(const Params &p, uint32_t it) {
    return BfsOp{p.val, p.parent, p.visited, it + 1};
}

// Refresh the BFS visited bitmap from the level array: one ballot per 64
// consecutive vertices, coalesced reads, one plain word store per 32
// vertices.  Readers may see old or new words concurrently; both only ever
// mark visited vertices, so any mix is a valid filter.
__device__ __forceinline__ void refresh_bitmap(const Params &p) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t v = base + threadIdx.x;
        const bool vis = v < n && p.val[v] != kInf;
        const unsigned long long m = __ballot(vis);
        const int lane = lane_id();
        const uint32_t v0 = v - static_cast<uint32_t>(lane);  // first vertex of this wavefront
        if (lane == 0 && v0 < n) p.visited[v0 >> 5] = static_cast<uint32_t>(m);
        if (lane == 32 && v < n) p.visited[v >> 5] = static_cast<uint32_t>(m >> 32);
    }
}

template <class Op>
__device__ __forceinline__ void level_prologue(const Params &, uint32_t) {}

template <>
__device__ __forceinline__ void level_prologue<BfsOp>(const Params &p, uint32_t cnt_in) {
    if (p.visited && cnt_in >= p.t_bitmap) refresh_bitmap(p);
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
    s->reserved = 0;
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

// Trace of invocation `it` (only when a trace buffer is given): edges this
// workgroup scanned, and the number of vertices deferred to the grid tier.
__device__ __forceinline__ void trace_level(const Params &p, uint32_t it, unsigned long long edges,
                                            const unsigned long long *hub_ctr) {
    __shared__ unsigned long long s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    if (edges) atomicAdd(&s_sum, edges);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&p.trace[4 * it + 2], s_sum);
        if (blockIdx.x == 0) p.trace[4 * it + 3] = hub_ctr[0] >> 40;
    }
}

// Grid tier of invocation `it`: read the settled deferred-vertex counter.
__device__ __forceinline__ void hub_counts(unsigned long long hc, uint32_t hub_cap, uint32_t &nh,
                                           uint32_t &nchunks) {
    nh = min(static_cast<uint32_t>(hc >> 40), hub_cap);
    nchunks = static_cast<uint32_t>(hc & ((1ull << 40) - 1));
}

// ---------------------------------------------------------------------------
// The outlined Iterate loop: one cooperative launch runs every invocation.
// An invocation that deferred vertices to the grid tier has two barriers
// (after phase A, after phase B); any other has one.
// ---------------------------------------------------------------------------
template <int B, class Op>
__global__ __launch_bounds__(B) void persistent_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    Ctrl *ctrl = p.ctrl;
    WaveQueue<kQueueCap> wq{sm.queue[wid], 0};
    BarrierState bs{0u, p.wd_ticks};
    unsigned long long edges = 0;
    const int32_t *in = p.wl0;
    int32_t *out = p.wl1;
    uint32_t it = 0;
    unsigned long long items = 0;
    uint32_t max_frontier = 0;

    for (;; ++it) {
        uint32_t cnt_in = load_agent(&ctrl->cnt[it % 3]);
        if (cnt_in > p.cap) cnt_in = p.cap;  // overflowed pushes were dropped (error set)
        if (cnt_in == 0) break;
        if (it >= p.max_iter) {
            if (blockIdx.x == 0 && tid == 0) set_error(ctrl, kErrIterLimit, false);
            break;
        }
        items += cnt_in;
        max_frontier = max(max_frontier, cnt_in);
        if (blockIdx.x == 0 && tid == 0) {
            store_agent(&ctrl->cnt[(it + 2) % 3], 0u);
            __hip_atomic_store(&ctrl->hub[(it + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (4 * it + 3 < p.trace_len) {
                p.trace[4 * it] = wall_clock64();
                p.trace[4 * it + 1] = cnt_in;
                p.trace[4 * it + 2] = 0;
                p.trace[4 * it + 3] = 0;
            }
        }
        const unsigned long long edges_before = edges;
        const Sink sk{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl};
        unsigned long long *hub_ctr = &ctrl->hub[it % 3];
        level_prologue<Op>(p, cnt_in);
        const Op op = make_op<Op>(p, it);
        expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, wq, sk,
                      p.t_wave, p.t_block, p.t_grid, p.hub_v, p.hub_base, p.hub_cap, hub_ctr, edges);
        block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, sk.cnt_out, out, p.cap, ctrl);
        if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag)) break;
        if (p.t_grid > 0) {
            // uniform: every workgroup reads the same settled counter
            uint32_t nh, nchunks;
            hub_counts(__hip_atomic_load(hub_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), p.hub_cap,
                       nh, nchunks);
            if (nh > 0) {
                expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, op, sm, wq, sk);
                block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, sk.cnt_out, out, p.cap, ctrl);
                if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag)) break;
            }
        }
        if (4 * it + 3 < p.trace_len) trace_level(p, it, edges - edges_before, hub_ctr);
        const int32_t *t = in;
        in = out;
        out = const_cast<int32_t *>(t);
    }

    // statistics and completion
    add_block_total<B>(edges, &ctrl->edges);
    if (tid == 0) {
        if (blockIdx.x == 0) {
            if (4 * it < p.trace_len) p.trace[4 * it] = wall_clock64();
            ctrl->iterations = it;
            ctrl->items = items;
            ctrl->max_frontier = max_frontier;
            ctrl->grid = static_cast<int32_t>(gridDim.x);
            ctrl->block = B;
        }
        const uint32_t prev = __hip_atomic_fetch_add(&ctrl->done, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            publish_stats(p);
        }
    }
}

// ---------------------------------------------------------------------------
// Un-outlined form: invocation `p.it` is one launch of level_kernel (phase
// A) and one of hub_level_kernel (phase B, returns at once when nothing was
// deferred); the host reads the outgoing count back after each invocation
// and decides whether to launch the next one.
// ---------------------------------------------------------------------------
template <int B, class Op>
__global__ __launch_bounds__(B) void level_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    Ctrl *ctrl = p.ctrl;
    const uint32_t it = p.it;
    WaveQueue<kQueueCap> wq{sm.queue[wid], 0};
    unsigned long long edges = 0;
    const int32_t *in = (it & 1u) ? p.wl1 : p.wl0;
    int32_t *out = (it & 1u) ? p.wl0 : p.wl1;
    uint32_t cnt_in = ctrl->cnt[it % 3];
    if (cnt_in > p.cap) cnt_in = p.cap;
    const Sink sk{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl};
    if (blockIdx.x == 0 && tid == 0 && 4 * it + 3 < p.trace_len) {
        p.trace[4 * it] = wall_clock64();
        p.trace[4 * it + 1] = cnt_in;
    }
    level_prologue<Op>(p, cnt_in);
    const Op op = make_op<Op>(p, it);
    expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, wq, sk, p.t_wave,
                  p.t_block, p.t_grid, p.hub_v, p.hub_base, p.hub_cap, &ctrl->hub[it % 3], edges);
    block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, sk.cnt_out, out, p.cap, ctrl);
    add_block_total<B>(edges, &ctrl->edges);
    if (tid == 0 && blockIdx.x == 0) {
        ctrl->cnt[(it + 2) % 3] = 0;
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
    WaveQueue<kQueueCap> wq{sm.queue[wid], 0};
    int32_t *out = (it & 1u) ? p.wl0 : p.wl1;
    const Sink sk{&ctrl->cnt[(it + 1) % 3], out, p.cap, ctrl};
    const Op op = make_op<Op>(p, it);
    expand_hubs<B, Op>(nh, nchunks, p.hub_v, p.hub_base, p.row_ptr, p.col, op, sm, wq, sk);
    block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, sk.cnt_out, out, p.cap, ctrl);
}

// Host-loop epilogue and the iteration-limit check of the un-outlined form.
__global__ void finish_kernel(Params p, int hit_limit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t it = p.ctrl->iterations;
        if (4 * it < p.trace_len) p.trace[4 * it] = wall_clock64();
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
    WaveQueue<kQueueCap> wq{sm.queue[wid], 0};
    unsigned long long edges = 0;
    const SsspParentOp op{p.val, p.w, p.parent, p.src};
    const Sink sk{nullptr, nullptr, 0u, p.ctrl};
    expand<B, SsspParentOp>(nullptr, static_cast<uint32_t>(p.n), static_cast<uint32_t>(p.n), p.row_ptr,
                            p.col, op, sm, wq, sk, p.t_wave, p.t_block, 0, nullptr, nullptr, 0u, nullptr,
                            edges);
}

// On-device CSR validation: row_ptr[0] == 0, monotone, row_ptr[n] == m,
// col in [0, n), w >= 1.  Sets *bad to 1 on any violation.
__global__ void validate_kernel(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col,
                                const uint32_t *w, uint32_t *bad) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (tid == 0 && (row_ptr[0] != 0 || static_cast<int64_t>(row_ptr[n]) != m)) atomicOr(bad, 1u);
    for (uint32_t v = tid; v < static_cast<uint32_t>(n); v += stride)
        if (row_ptr[v + 1] < row_ptr[v]) atomicOr(bad, 1u);
    for (uint64_t e = tid; e < static_cast<uint64_t>(m); e += stride) {
        const int32_t d = col[e];
        if (d < 0 || d >= n) atomicOr(bad, 1u);
        if (w && w[e] == 0u) atomicOr(bad, 1u);
    }
}

}  // namespace irgl
