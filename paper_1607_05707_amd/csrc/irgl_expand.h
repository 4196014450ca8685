// Frontier expansion: the outer ForAll over the incoming worklist with
// nested edge parallelism for the inner ForAll (workgroup / wavefront /
// prefix-sum tiers plus the grid tier), the staged cooperative pushes, and
// the SSSP far -> near transfer.
#pragma once

#include "irgl_ops.h"

namespace irgl {

// Where one invocation's pushes go.
struct Sink {
    uint32_t *cnt_out;
    int32_t *out;
    uint32_t cap;
    Ctrl *ctrl;
    uint32_t *min_out;  // far list: running lower bound of listed distances
};

// The wavefront's staging queues and where they drain to.
struct Pushers {
    WaveQueue<kQueueCap> nq;  // outgoing worklist (near)
    WaveQueue<kQueueCap> fq;  // SSSP far list
    Sink sk;
    Sink skf;
    uint32_t fmin;            // this lane's far-list lower bound since the last drain
    const int32_t *deg_rp;    // BFS direction choice: row offsets to sum pushed degrees, or null
    unsigned long long *mf_out;
    unsigned long long mf;    // this lane's sum of out-degrees of pushed vertices
    uint32_t tries = 0;       // this lane's claim atomics (trace statistics)
    uint32_t wins = 0;        // ... and the successful ones
    WaveQueue<kHeavyQ> hq{nullptr, 0};  // SSSP heavy list of the current bucket
    Sink skh{};               // its sink (cnt_out null: no heavy list in this invocation)
    unsigned long long hdeg = 0;           // this lane's heavy out-degrees of listed vertices
    unsigned long long *hsum_out = nullptr;  // ... drained into this per-bucket counter
    uint32_t hminv = kInf;                 // this lane's smallest distance of an expanded vertex
    uint32_t *hmin_out = nullptr;          // ... drained into this per-bucket minimum
    __device__ __forceinline__ void near(bool p, int item) {
        nq.push(p, item, sk.cnt_out, sk.out, sk.cap, sk.ctrl);
    }
    __device__ __forceinline__ void far(bool p, int item) {
        fq.push(p, item, skf.cnt_out, skf.out, skf.cap, skf.ctrl);
    }
    // All 64 lanes call it (uniform call site); does nothing without a list.
    __device__ __forceinline__ void heavy(bool p, int item) {
        if (skh.cnt_out) hq.push(p, item, skh.cnt_out, skh.out, skh.cap, skh.ctrl);
    }
};

// Row range an operator relaxes for vertex v (default: the whole row).
template <class Op>
__device__ __forceinline__ void op_range(const Op &, const int32_t *__restrict__ rp, int v, int &r0, int &r1) {
    r0 = rp[v];
    r1 = rp[v + 1];
}
template <>
__device__ __forceinline__ void op_range<SsspOp>(const SsspOp &op, const int32_t *__restrict__ rp, int v, int &r0,
                                                 int &r1) {
    if (!op.split) {
        r0 = rp[v];
        r1 = rp[v + 1];
    } else if (op.heavy) {
        r0 = op.split[v];
        r1 = rp[v + 1];
    } else {
        r0 = rp[v];
        r1 = op.split[v];
    }
}

// Pop-time decision for vertex v with value val (default: expand it).
// SSSP: a vertex whose distance has not changed since its last expansion is
// not expanded again (every edge was relaxed with this distance, or a
// smaller one no longer current is impossible: distances only fall); an
// expanded vertex is listed once per bucket for the heavy pass (*hpush).
template <class Op>
__device__ __forceinline__ bool op_pop(const Op &, int, uint32_t, bool &) {
    return true;
}
template <>
__device__ __forceinline__ bool op_pop<SsspOp>(const SsspOp &op, int v, uint32_t val, bool &hpush) {
    if (op.expd) {
        if (op.expd[v] == val) return false;
        op.expd[v] = val;
    }
    if (op.hstamp && op.hstamp[v] != op.bucket) {
        op.hstamp[v] = op.bucket;
        hpush = true;
    }
    return true;
}

// Heavy out-degree of vertex v (the part of its row a heavy pass scans).
template <class Op>
__device__ __forceinline__ unsigned long long op_heavy_degree(const Op &, const int32_t *__restrict__, int) {
    return 0ull;
}
template <>
__device__ __forceinline__ unsigned long long op_heavy_degree<SsspOp>(const SsspOp &op, const int32_t *__restrict__ rp,
                                                                       int v) {
    return op.split ? static_cast<unsigned long long>(rp[v + 1] - op.split[v]) : 0ull;
}

// Workgroup-wide drain of both queues (all threads call it).
template <int B, class Op, class S>
__device__ __forceinline__ void drain_all(Pushers &pu, S &sm) {
    block_drain<B, kQueueCap>(pu.nq, sm.fill, &sm.base, pu.sk.cnt_out, pu.sk.out, pu.sk.cap, pu.sk.ctrl);
    if (pu.deg_rp) {
        // one atomicAdd per wavefront: out-degree sum of the pushed vertices
        unsigned long long x = pu.mf;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) x += __shfl_xor(x, d, kWave);
        if (lane_id() == 0 && x) atomicAdd(pu.mf_out, x);
        pu.mf = 0;
    }
    if (Op::kFar && pu.skh.cnt_out)  // uniform: the same sink for the whole team
        block_drain<B, kHeavyQ>(pu.hq, sm.fill, &sm.base, pu.skh.cnt_out, pu.skh.out, pu.skh.cap, pu.skh.ctrl);
    if (Op::kFar && pu.hsum_out) {  // uniform; one atomicAdd and one atomicMin per wavefront
        unsigned long long x = pu.hdeg;
        uint32_t mn = pu.hminv;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            x += __shfl_xor(x, d, kWave);
            mn = min(mn, static_cast<uint32_t>(__shfl_xor(mn, d, kWave)));
        }
        if (lane_id() == 0 && x) atomicAdd(pu.hsum_out, x);
        if (lane_id() == 0 && mn != kInf) atomicMin(pu.hmin_out, mn);
    }
    // also where nothing was drained (a heavy pass expands settled vertices):
    // their values must not reach the next bucket's minimum
    pu.hdeg = 0;
    pu.hminv = kInf;
    if (Op::kFar) {
        block_drain<B, kQueueCap>(pu.fq, sm.fill, &sm.base, pu.skf.cnt_out, pu.skf.out, pu.skf.cap,
                                  pu.skf.ctrl);
        // one atomicMin per workgroup for the far-list lower bound
        uint32_t m = pu.fmin;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) m = min(m, static_cast<uint32_t>(__shfl_xor(m, d, kWave)));
        __syncthreads();  // every wave has finished reading sm.fill in block_drain
        if (lane_id() == 0) sm.fill[threadIdx.x / kWave] = static_cast<int>(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t bm = kInf;
            for (int k = 0; k < B / kWave; ++k) bm = min(bm, static_cast<uint32_t>(sm.fill[k]));
            if (bm != kInf) atomicMin(pu.skf.min_out, bm);
        }
        __syncthreads();
        pu.fmin = kInf;
    }
}

// Relax U edges of one lane and push the survivors (all 64 lanes call it).
template <class Op>
__device__ __forceinline__ void relax_and_push(const Op &op, const int32_t *__restrict__ col,
                                               const int (&e)[Op::kU], bool (&act)[Op::kU], const int (&sv)[Op::kU],
                                               const uint32_t (&sval)[Op::kU], Pushers &pu) {
    int d[Op::kU];
    bool far[Op::kU];
#pragma unroll
    for (int k = 0; k < Op::kU; ++k) {
        d[k] = act[k] ? col[e[k]] : 0;
        far[k] = false;
    }
    op.relax(e, d, sv, sval, act, far, pu.fmin, pu.tries, pu.wins);
    if (!Op::kFar && pu.deg_rp) {
#pragma unroll
        for (int k = 0; k < Op::kU; ++k)
            if (act[k]) pu.mf += static_cast<unsigned long long>(pu.deg_rp[d[k] + 1] - pu.deg_rp[d[k]]);
    }
    if (Op::kPush) {
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) pu.near(act[k], d[k]);
    }
    if (Op::kFar) {
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) pu.far(far[k], d[k]);
    }
}

// A group of `width` lanes (lane index `li` in it) strides the range
// [r0, r1) of vertex sv, U edges per lane per round.  The trip count is
// uniform across the group.
template <class Op>
__device__ __forceinline__ void stride_range(const Op &op, const int32_t *__restrict__ col, int r0,
                                             int r1, int sv, uint32_t sval, int li, int width,
                                             Pushers &pu) {
    int svs[Op::kU];
    uint32_t svals[Op::kU];
#pragma unroll
    for (int k = 0; k < Op::kU; ++k) {
        svs[k] = sv;
        svals[k] = sval;
    }
    for (int e0 = r0; e0 < r1; e0 += width * Op::kU) {
        int e[Op::kU];
        bool act[Op::kU];
#pragma unroll
        for (int k = 0; k < Op::kU; ++k) {
            e[k] = e0 + k * width + li;
            act[k] = e[k] < r1;
        }
        relax_and_push(op, col, e, act, svs, svals, pu);
    }
}

// ---------------------------------------------------------------------------
// Phase A of one invocation: nested-parallel expansion of the incoming
// worklist.  `in == nullptr` means the identity worklist 0..cnt_in-1.
// Vertices of out-degree >= t_grid (t_grid > 0; t_block for a small
// worklist) are appended to the grid-tier list (hub_v / hub_base, counted by
// *hub_ctr) instead of being expanded here.  Every thread of every workgroup
// must call it (it may synchronise the workgroup).
// ---------------------------------------------------------------------------
// Small worklists: a range of at least kSmallDefer entries goes to the grid
// tier (one workgroup per chunk) rather than to its one wavefront, which
// would walk it in ceil(deg / (64 U)) dependent rounds.  The first BFS
// invocations on R-MAT (tens of items, tens of thousands of entries) then
// end with the hub phase, not with one wavefront's long walk: RMAT-22 BFS
// 368 against 386 us per query at B (1024), RMAT-21 304 against 314; SSSP
// and the road grid unchanged; 128 and 512 within 1% of 256.
constexpr int kSmallDefer = 256;

template <int B, class Op>
__device__ __forceinline__ void expand(const int32_t *__restrict__ in, uint32_t cnt_in, uint32_t n,
                                       const int32_t *__restrict__ row_ptr,
                                       const int32_t *__restrict__ col, const Op &op, Smem<B> &sm,
                                       Pushers &pu, int t_wave,
                                       int t_block, int t_grid, int32_t *hub_v, uint32_t *hub_base,
                                       uint32_t hub_cap, unsigned long long *hub_ctr,
                                       unsigned long long &edges, Team tm, uint32_t *tile_ctr) {
    constexpr int NW = B / kWave;
    constexpr int kChunk = B * Op::kU;
    static_assert(Op::kU <= kUMax, "the gather window in LDS holds B * kUMax slots");
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wid = tid / kWave;
    const uint32_t stride = tm.size * B;

    // Small worklist (no more items than wavefronts in the team): one item per
    // wavefront, dealt across workgroups first, so that the ranges of a few
    // items are not walked one after another by a few workgroups.  Ranges of
    // kSmallDefer or more entries go to the grid tier (when its list is full,
    // to the wavefront after all).
    if (t_grid > 0 && cnt_in <= tm.size * NW) {
        const uint32_t i = static_cast<uint32_t>(wid) * tm.size + tm.id;
        if (i >= cnt_in) return;  // uniform across the wavefront
        int v = in ? in[i] : static_cast<int>(i);
        int r0 = 0, r1 = 0;
        uint32_t val = 0;
        if (static_cast<uint32_t>(v) >= n) {  // never expected: a corrupt worklist entry
            if (lane == 0) set_error(pu.sk.ctrl, kErrInternal, false);
            return;
        }
        val = op.vertex_value(v);
        bool hp = false, ex = false;
        if (op.active(val) && op_pop(op, v, val, hp)) {
            op_range(op, row_ptr, v, r0, r1);
            ex = true;
        }
        pu.heavy(hp && lane == 0, v);
        if (hp && lane == 0) pu.hdeg += op_heavy_degree(op, row_ptr, v);
        if (ex) pu.hminv = min(pu.hminv, val);  // every expansion, listed or not
        const int deg = r1 - r0;
        if (lane == 0) edges += static_cast<unsigned long long>(deg);
        if (deg >= kSmallDefer) {  // a range of several wavefront rounds goes to the grid tier
            int listed = 0;
            if (lane == 0) {
                const unsigned long long old = atomicAdd(
                    hub_ctr, (1ull << 40) | static_cast<unsigned long long>((deg + kChunk - 1) / kChunk));
                const uint32_t slot = static_cast<uint32_t>(old >> 40);
                if (slot < hub_cap) {
                    hub_v[slot] = v;
                    hub_base[slot] = static_cast<uint32_t>(old & ((1ull << 40) - 1));
                    listed = 1;
                }
            }
            if (__shfl(listed, 0, kWave)) return;
        }
        stride_range(op, col, r0, r1, v, val, lane, kWave, pu);
        return;
    }

    // A worklist with fewer items than the team has threads leaves whole
    // workgroups without a tile while others walk long ranges: then every
    // range of a round (B edges) or more goes to the balanced grid tier.
    if (t_grid > B && cnt_in < stride) t_grid = B;
    // Tiles of B items: first one per workgroup, then (with tile_ctr) taken
    // from a shared counter, so that workgroups with light tiles take more.
    // SSSP: such a worklist would fill only cnt_in / B workgroups, and one
    // tile of B medium-degree vertices (a light phase just after the first
    // hubs) then keeps one workgroup busy for a tenth of the query; its tiles
    // hold ceil(cnt_in / team size) items instead (at least 128), so that
    // every workgroup takes a share.  Consecutive items stay on consecutive
    // threads (pushes of one wavefront are often neighbouring vertices).
    const uint32_t tsz = (Op::kFar && cnt_in < stride)
                             ? min(static_cast<uint32_t>(B), max(128u, (cnt_in + tm.size - 1) / tm.size))
                             : static_cast<uint32_t>(B);
    uint32_t tile = tm.id;
    for (;;) {
        const uint32_t base = tile * tsz;
        if (base >= cnt_in) break;  // uniform across the workgroup
        const uint32_t i = base + tid;
        int v = -1, r0 = 0, r1 = 0;
        uint32_t val = 0;
        bool hp = false, ex = false;
        if (static_cast<uint32_t>(tid) < tsz && i < cnt_in) {
            v = in ? in[i] : static_cast<int>(i);
            if (static_cast<uint32_t>(v) >= n) {  // never expected: a corrupt worklist entry
                set_error(pu.sk.ctrl, kErrInternal, false);
                v = -1;
            } else {
                val = op.vertex_value(v);
                if (op.active(val) && op_pop(op, v, val, hp)) {
                    op_range(op, row_ptr, v, r0, r1);
                    ex = true;
                }
            }
        }
        pu.heavy(hp, v);
        if (hp) pu.hdeg += op_heavy_degree(op, row_ptr, v);
        if (ex) pu.hminv = min(pu.hminv, val);  // every expansion, listed or not
        int deg = r1 - r0;
        edges += static_cast<unsigned long long>(deg);

        // Tier 0: defer the largest ranges to the grid-wide phase.  One packed
        // atomicAdd per wavefront reserves list slots and chunk numbers for all
        // its deferring lanes, in lane order, so slot order is chunk order.
        if (t_grid > 0) {
            const bool defer = deg >= t_grid;
            const unsigned long long dm = __ballot(defer);
            if (dm) {
                const int chunks = defer ? (deg + kChunk - 1) / kChunk : 0;
                const int cincl = wave_inclusive_scan(chunks);
                const int ctotal = __shfl(cincl, kWave - 1, kWave);
                unsigned long long old = 0;
                if (lane == 0)
                    old = atomicAdd(hub_ctr, (static_cast<unsigned long long>(__popcll(dm)) << 40) |
                                                 static_cast<unsigned long long>(ctotal));
                old = __shfl(old, 0, kWave);
                if (defer) {
                    const uint32_t slot = static_cast<uint32_t>(old >> 40) + lane_rank(dm);
                    if (slot < hub_cap) {
                        hub_v[slot] = v;
                        hub_base[slot] = static_cast<uint32_t>(old & ((1ull << 40) - 1)) +
                                         static_cast<uint32_t>(cincl - chunks);
                        deg = 0;
                    }  // else: list full, expanded here (cannot happen: cap >= m / t_grid + 1)
                }
            }
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
            stride_range(op, col, sm.big_r0, sm.big_r1, sm.big_v, sm.big_val, tid, B, pu);
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
            stride_range(op, col, w0, w1, wv, wval, lane, kWave, pu);
        }

        // Tier 3: the remaining ranges of the workgroup are concatenated by an
        // exclusive prefix sum and dealt to the lanes in rounds of B*U edges,
        // every round full: slot s belongs to the last thread whose range
        // starts at or before s (a binary search over the scan in LDS), so a
        // workgroup needs ceil(total / (B*U)) rounds whatever the degree mix.
        const int incl = wave_inclusive_scan(deg);
        if (lane == kWave - 1) sm.wsum[wid] = incl;
        __syncthreads();
        int total = 0, wpre = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int s = sm.wsum[k];
            wpre += (k < wid) ? s : 0;
            total += s;
        }
        sm.gstart[tid] = wpre + incl - deg;
        sm.gr0[tid] = r0;
        sm.vtx[tid] = v;
        sm.vval[tid] = val;
        __syncthreads();
        for (int done = 0; done < total; done += kChunk) {
            int e[Op::kU], sv[Op::kU];
            uint32_t sval[Op::kU];
            bool act[Op::kU];
#pragma unroll
            for (int k = 0; k < Op::kU; ++k) {
                const int slot = done + k * B + tid;
                act[k] = slot < total;
                int o = 0;
#pragma unroll
                for (int step = B / 2; step > 0; step >>= 1)
                    if (sm.gstart[o + step] <= slot) o += step;
                e[k] = act[k] ? sm.gr0[o] + (slot - sm.gstart[o]) : 0;
                sv[k] = sm.vtx[o];
                sval[k] = sm.vval[o];
            }
            relax_and_push(op, col, e, act, sv, sval, pu);
        }
        if (tile_ctr) {
            if (tid == 0) sm.tile = tm.size + atomicAdd(tile_ctr, 1u);
        }
        __syncthreads();  // the scan arrays are rewritten by the next tile; sm.tile is set
        tile = tile_ctr ? sm.tile : tile + tm.size;
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
                                            Pushers &pu, Team tm) {
    constexpr int kChunk = B * Op::kU;
    const unsigned long long G = tm.size;
    const uint32_t lo = static_cast<uint32_t>(nchunks * static_cast<unsigned long long>(tm.id) / G);
    const uint32_t hi = static_cast<uint32_t>(nchunks * static_cast<unsigned long long>(tm.id + 1) / G);
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
        int r0, r1;
        op_range(op, row_ptr, v, r0, r1);
        const uint32_t nch = static_cast<uint32_t>((r1 - r0 + kChunk - 1) / kChunk);
        const uint32_t c_end = min(hi, cb + nch);
        const int e_lo = r0 + static_cast<int>((c - cb) * kChunk);
        const int e_hi = min(r1, r0 + static_cast<int>((c_end - cb) * kChunk));
        const uint32_t val = op.vertex_value(v);
        stride_range(op, col, e_lo, e_hi, v, val, threadIdx.x, B, pu);
        c = c_end;
        ++h;
    }
}

// ---------------------------------------------------------------------------
// SSSP far -> near transfer after the threshold rises from t_old to t_new.
// A listed vertex whose distance is already below t_old was expanded at that
// distance by a near invocation (dropped); one below t_new joins the next
// worklist; the rest stays listed.  Called by all threads of every workgroup.
// ---------------------------------------------------------------------------
// A vertex moved to the worklist claims its push stamp for invocation `it`,
// so that a relaxation in the same invocation cannot list it a second time.
template <int B>
__device__ __forceinline__ void far_transfer(const int32_t *far_in, uint32_t far_n, uint32_t n,
                                             uint32_t t_old, uint32_t t_new, const uint32_t *dist,
                                             uint32_t *far_flag, uint32_t *stamp, uint32_t it, Pushers &pu,
                                             Team tm) {
    const uint32_t stride = tm.size * B;
    for (uint32_t base = tm.id * B; base < far_n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        int v = 0;
        bool to_near = false, keep = false;
        if (i < far_n) {
            v = far_in[i];
            if (static_cast<uint32_t>(v) >= n) {  // never expected: a corrupt list entry
                set_error(pu.sk.ctrl, kErrInternal, false);
                v = 0;
            } else {
                const uint32_t dv = dist[v];
                if (dv < t_new) far_flag[v] = 0u;
                to_near = dv >= t_old && dv < t_new;
                if (to_near) to_near = atomicExch(&stamp[v], it) != it;
                keep = dv >= t_new;
                if (keep) pu.fmin = min(pu.fmin, dv);
            }
        }
        pu.near(to_near, v);
        pu.far(keep, v);
    }
}

}  // namespace irgl
