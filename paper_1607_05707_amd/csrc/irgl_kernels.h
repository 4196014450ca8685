// gfx950 kernels of the data-driven BFS/SSSP hot path.
//
//   * Frontier expansion: the outer ForAll over the incoming worklist
//     (Section 3.1: consecutive items on consecutive lanes) with nested edge
//     parallelism for the inner ForAll over graph.edges(n) (Sections 4.1 and
//     4.3): workgroup / wavefront / prefix-sum-gather tiers by out-degree.
//   * Relax operators: the BFS check-and-label of the Section 4.1 listing made
//     exactly-once with a compare-and-swap; the SSSP "distance improved" test
//     with atomicMin and a per-invocation push stamp.
//   * The outlined Iterate loop (Sections 4.2 and 4.3): one persistent,
//     co-resident grid that runs every invocation, separated by the grid
//     barrier, swapping the in/out worklists each time.
//   * The un-outlined form: one launch per invocation.
//   * Initialisation (the worklist initializer [src]) and the SSSP parent pass.
#pragma once

#include "irgl_device.h"

namespace irgl {

constexpr int kQueueCap = 256;  // LDS staging entries per wavefront

// Shared-memory layout of the frontier kernels for workgroup size B.
template <int B>
struct Smem {
    static constexpr int NW = B / kWave;
    int gather_edge[B];      // edge index of each slot of the current gather window
    int gather_owner[B];     // thread whose vertex owns that edge
    int vtx[B];              // popped vertex of each thread
    uint32_t vval[B];        // its per-vertex value (SSSP distance at pop)
    int wsum[NW];            // per-wavefront degree sums for the workgroup scan
    int fill[NW];            // per-wavefront queue fill at the workgroup drain
    int queue[NW][kQueueCap];
    int owner;               // workgroup-tier vertex owner
    int big_r0, big_r1, big_v;
    uint32_t big_val;
    uint32_t base;
    int flag;
    uint32_t cnt_in;
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
    Ctrl *ctrl;
    Stats *dstats;        // optional
    uint32_t cap;         // worklist capacity
    uint32_t max_iter;
    int32_t t_wave;
    int32_t t_block;
    int32_t src;
    uint32_t it;          // host-loop mode: the invocation to run
    unsigned long long wd_ticks;
    const volatile int32_t *abort_flag;
};

// ---------------------------------------------------------------------------
// Relax operators.  relax() is called once per scanned edge e = (sv -> d);
// it returns true when d must be pushed on the outgoing worklist.
// ---------------------------------------------------------------------------
struct BfsOp {
    static constexpr bool kPush = true;
    uint32_t *level;
    int32_t *parent;
    uint32_t next;  // label of vertices found in this invocation
    __device__ __forceinline__ uint32_t vertex_value(int) const { return 0u; }
    __device__ __forceinline__ bool active(uint32_t) const { return true; }
    __device__ __forceinline__ bool relax(int, int d, int sv, uint32_t) const {
        // A plain (possibly stale) load filters out most visited vertices;
        // stale values can only read INF, and the CAS below decides.
        if (level[d] != kInf) return false;
        if (atomicCAS(&level[d], kInf, next) != kInf) return false;
        if (parent) parent[d] = sv;
        return true;
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
    __device__ __forceinline__ bool relax(int e, int d, int, uint32_t dv) const {
        const uint32_t nd = dv + w[e];
        if (nd < dv || nd == kInf) {  // the sum does not fit below the INF sentinel
            set_error(ctrl, kErrOverflow, false);
            return false;
        }
        if (nd >= dist[d]) return false;
        const uint32_t old = atomicMin(&dist[d], nd);
        if (nd >= old) return false;
        // push d at most once per invocation
        if (stamp[d] == it) return false;
        return atomicExch(&stamp[d], it) != it;
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
    __device__ __forceinline__ bool relax(int e, int d, int sv, uint32_t dv) const {
        if (d != src && dv + w[e] == dist[d] && dv + w[e] >= dv)
            atomicMin(reinterpret_cast<uint32_t *>(&parent[d]), static_cast<uint32_t>(sv));
        return false;
    }
};

// ---------------------------------------------------------------------------
// Nested-parallel expansion of one invocation's incoming worklist.
// `in == nullptr` means the identity worklist 0..cnt_in-1.  Every thread of
// every workgroup must call it (it synchronises the workgroup).
// ---------------------------------------------------------------------------
template <int B, class Op>
__device__ __forceinline__ void expand(const int32_t *__restrict__ in, uint32_t cnt_in, uint32_t n,
                                       const int32_t *__restrict__ row_ptr,
                                       const int32_t *__restrict__ col, const Op &op, Smem<B> &sm,
                                       WaveQueue<kQueueCap> &wq, uint32_t *cnt_out, int32_t *out,
                                       uint32_t cap, Ctrl *ctrl, int t_wave, int t_block,
                                       unsigned long long &edges) {
    constexpr int NW = B / kWave;
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
                set_error(ctrl, kErrInternal, false);
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
            const int b0 = sm.big_r0, b1 = sm.big_r1, bv = sm.big_v;
            const uint32_t bval = sm.big_val;
            for (int e0 = b0; e0 < b1; e0 += B) {
                const int e = e0 + tid;
                bool p = false;
                int d = 0;
                if (e < b1) {
                    d = col[e];
                    p = op.relax(e, d, bv, bval);
                }
                if (Op::kPush) wq.push(p, d, cnt_out, out, cap, ctrl);
            }
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
            for (int e0 = w0; e0 < w1; e0 += kWave) {
                const int e = e0 + lane;
                bool p = false;
                int d = 0;
                if (e < w1) {
                    d = col[e];
                    p = op.relax(e, d, wv, wval);
                }
                if (Op::kPush) wq.push(p, d, cnt_out, out, cap, ctrl);
            }
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
        for (int done = 0; done < total; done += B) {
            const int lo = max(excl, done);
            const int hi = min(excl + deg, done + B);
            for (int k = lo; k < hi; ++k) {
                sm.gather_edge[k - done] = r0 + (k - excl);
                sm.gather_owner[k - done] = tid;
            }
            __syncthreads();
            bool p = false;
            int d = 0;
            if (tid < total - done) {
                const int e = sm.gather_edge[tid];
                const int o = sm.gather_owner[tid];
                d = col[e];
                p = op.relax(e, d, sm.vtx[o], sm.vval[o]);
            }
            if (Op::kPush) wq.push(p, d, cnt_out, out, cap, ctrl);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation: val = INF except val[src] = 0; parent = -1 except
// parent[src] = src; stamps = INF; in = [src]; counters and stats cleared.
// ---------------------------------------------------------------------------
__global__ void init_kernel(Params p, int with_stamp) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool s = static_cast<int>(i) == p.src;
        p.val[i] = s ? 0u : kInf;
        if (p.parent) p.parent[i] = s ? p.src : -1;
        if (with_stamp) p.stamp[i] = kInf;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl *c = p.ctrl;
        c->cnt[0] = 1;
        c->cnt[1] = 0;
        c->cnt[2] = 0;
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
__device__ __forceinline__ BfsOp make_op<BfsOp>(const Params &p, uint32_t it) {
    return BfsOp{p.val, p.parent, it + 1};
}

template <>
__device__ __forceinline__ SsspOp make_op<SsspOp>(const Params &p, uint32_t it) {
    return SsspOp{p.val, p.w, p.stamp, it, p.ctrl};
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

// ---------------------------------------------------------------------------
// The outlined Iterate loop: one cooperative launch runs every invocation.
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
        if (blockIdx.x == 0 && tid == 0) store_agent(&ctrl->cnt[(it + 2) % 3], 0u);
        uint32_t *cnt_out = &ctrl->cnt[(it + 1) % 3];
        const Op op = make_op<Op>(p, it);
        expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, wq, cnt_out, out, p.cap, ctrl,
                      p.t_wave, p.t_block, edges);
        block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, cnt_out, out, p.cap, ctrl);
        if (!grid_barrier(ctrl, bs, &sm.flag, p.abort_flag)) break;
        const int32_t *t = in;
        in = out;
        out = const_cast<int32_t *>(t);
    }

    // statistics and completion
    __shared__ unsigned long long s_edges;
    if (tid == 0) s_edges = 0;
    __syncthreads();
    atomicAdd(&s_edges, edges);
    __syncthreads();
    if (tid == 0) {
        atomicAdd(&ctrl->edges, s_edges);
        if (blockIdx.x == 0) {
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
// Un-outlined form: one launch per invocation `p.it`; the host reads the
// outgoing count back and decides whether to launch the next one.
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
    uint32_t *cnt_out = &ctrl->cnt[(it + 1) % 3];
    const Op op = make_op<Op>(p, it);
    expand<B, Op>(in, cnt_in, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, wq, cnt_out, out, p.cap, ctrl, p.t_wave,
                  p.t_block, edges);
    block_drain<B, kQueueCap>(wq, sm.fill, &sm.base, cnt_out, out, p.cap, ctrl);
    __shared__ unsigned long long s_edges;
    if (tid == 0) s_edges = 0;
    __syncthreads();
    atomicAdd(&s_edges, edges);
    __syncthreads();
    if (tid == 0) {
        atomicAdd(&ctrl->edges, s_edges);
        if (blockIdx.x == 0) {
            ctrl->cnt[(it + 2) % 3] = 0;
            ctrl->iterations = it + 1;
            ctrl->items += cnt_in;
            ctrl->max_frontier = max(ctrl->max_frontier, cnt_in);
            ctrl->grid = static_cast<int32_t>(gridDim.x);
            ctrl->block = B;
        }
    }
}

// Host-loop epilogue and the iteration-limit check of the un-outlined form.
__global__ void finish_kernel(Params p, int hit_limit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (hit_limit) set_error(p.ctrl, kErrIterLimit, false);
        publish_stats(p);
    }
}

// SSSP parent pass over the identity worklist of all n vertices.
template <int B>
__global__ __launch_bounds__(B) void sssp_parent_kernel(Params p) {
    __shared__ Smem<B> sm;
    const int wid = threadIdx.x / kWave;
    WaveQueue<kQueueCap> wq{sm.queue[wid], 0};
    unsigned long long edges = 0;
    const SsspParentOp op{p.val, p.w, p.parent, p.src};
    expand<B, SsspParentOp>(nullptr, static_cast<uint32_t>(p.n), static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm, wq,
                            nullptr, nullptr, 0u, p.ctrl, p.t_wave, p.t_block, edges);
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
