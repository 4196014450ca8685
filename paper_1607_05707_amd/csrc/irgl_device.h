// Device-side building blocks shared by every gfx950 kernel of the library:
// the control block that lives at the head of a query's workspace, wave64
// helpers, the cooperative (aggregated) worklist push and the grid-wide
// barrier of the outlined Iterate loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace irgl {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kWave = 64;

// Error codes written by the device (same values as the public irgl_status).
constexpr uint32_t kErrOverflow = 5;
constexpr uint32_t kErrAborted = 6;
constexpr uint32_t kErrWatchdog = 11;
constexpr uint32_t kErrIterLimit = 12;
constexpr uint32_t kErrInternal = 14;

// Control block at offset 0 of a query workspace.  Hot words sit on their own
// 128-byte lines so that polling one does not contend with updates of another.
constexpr int kBarGroups = 8;  // one arrival group per XCD (workgroup id mod 8)

struct alignas(128) Ctrl {
    // line 0: rotating worklist counters.  Invocation `it` pops cnt[it % 3]
    // items, pushes through cnt[(it + 1) % 3] and clears cnt[(it + 2) % 3],
    // which nobody reads again before the next barrier has passed.
    uint32_t cnt[3];
    uint32_t pad0a;
    // rotating grid-tier counters, packed (deferred vertices << 40 | chunks)
    unsigned long long hub[3];
    // rotating SSSP far-list counters (indexed by threshold raises so far)
    uint32_t far_cnt[3];
    // rotating SSSP lower bounds on the distances of far-listed vertices
    uint32_t far_min[3];
    // rotating BFS sums of out-degrees of the next frontier (direction choice)
    unsigned long long mf[3];
    // BFS: edges scanned by bottom-up invocations so far (grows, never reset)
    unsigned long long bu_scan;
    // rotating worklist-tile counters (tiles taken beyond each workgroup's first)
    uint32_t tile[3];
    // rotating ReduceAndReturn words of the topology-driven loop (one per invocation)
    uint32_t red[3];
    uint32_t pad0[2];
    // line 1: barrier generation (the only word waiting workgroups poll)
    uint32_t bar_gen;
    uint32_t pad1[31];
    // line 2: top-level barrier arrivals (one per group per barrier)
    unsigned long long bar_top;
    uint32_t pad2[30];
    // lines 3..10: per-group barrier arrivals
    struct alignas(128) Group {
        unsigned long long count;
        uint32_t pad[30];
    } bar_grp[kBarGroups];
    // line 11: errors.  `error` keeps the first code; `fatal` makes waiting
    // workgroups leave the barrier (watchdog, abort).
    uint32_t error;
    uint32_t fatal;
    uint32_t done;  // workgroups that have left the kernel
    uint32_t xmap_bad;  // a workgroup of this launch is not on XCD (id mod 8)
    uint32_t pad3[28];
    // line 12: statistics
    uint32_t iterations;
    uint32_t max_frontier;
    unsigned long long items;
    unsigned long long edges;
    int32_t grid;
    int32_t block;
    unsigned long long fedges;  // sum of out-degrees of every frontier
    // rotating SSSP sums of the heavy out-degrees of the listed vertices
    // (indexed by threshold raises so far): the edges a push heavy pass scans
    unsigned long long hsum[3];
    // rotating SSSP heavy-list counters (indexed by threshold raises so far)
    uint32_t hcnt[3];
    // rotating SSSP smallest distance of a vertex expanded in the bucket
    uint32_t hmin[3];
    // rotating (per invocation) SSSP flag: a pull heavy pass met a vertex it
    // leaves to the push pass
    uint32_t hbig[3];
    uint32_t pulls;  // SSSP heavy passes run as a pull
    uint32_t pad4[6];
};
static_assert(sizeof(Ctrl) == 13 * 128, "control block layout");

// Host-visible statistics (layout of irgl_stats).
struct Stats {
    int32_t status;
    uint32_t iterations;
    unsigned long long items;
    unsigned long long edges;
    uint32_t max_frontier;
    int32_t grid;
    int32_t block;
    uint32_t heavy_pulls;
    unsigned long long frontier_edges;
};

__device__ __forceinline__ void set_error(Ctrl *c, uint32_t code, bool fatal) {
    atomicCAS(&c->error, 0u, code);
    if (fatal) __hip_atomic_store(&c->fatal, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane (the lane's rank among the
// active predicates of its wavefront).
__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ int wave_inclusive_scan(int x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// ---------------------------------------------------------------------------
// Cooperative worklist push (cooperative conversion, Sections 3.5 and 4.2).
//
// Lanes holding an item to push form a ballot; the wavefront appends the
// items, in lane order, to its private staging queue in LDS.  A full queue is
// drained by the wavefront alone with ONE atomicAdd on the global out-counter
// and a contiguous copy; at the end of an invocation the whole workgroup
// drains the remainders of all its wavefronts with ONE atomicAdd.
// ---------------------------------------------------------------------------
template <int QCAP>
struct WaveQueue {
    int *q;     // this wavefront's LDS staging area, QCAP entries
    int n;      // wave-uniform fill level

    __device__ __forceinline__ void drain(uint32_t *cnt_out, int *out, uint32_t cap, Ctrl *ctrl) {
        if (n == 0) return;
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(cnt_out, static_cast<uint32_t>(n));
        base = __shfl(base, 0, kWave);
        __builtin_amdgcn_wave_barrier();
        if (base + static_cast<uint32_t>(n) > cap || base + static_cast<uint32_t>(n) < base) {
            if (lane_id() == 0) set_error(ctrl, kErrOverflow, false);
        }
        for (int j = lane_id(); j < n; j += kWave) {
            uint32_t dst = base + static_cast<uint32_t>(j);
            if (dst < cap && dst >= base) out[dst] = q[j];
        }
        __builtin_amdgcn_wave_barrier();
        n = 0;
    }

    // All 64 lanes must call push together (wave-uniform control flow).
    __device__ __forceinline__ void push(bool pred, int item, uint32_t *cnt_out, int *out,
                                         uint32_t cap, Ctrl *ctrl) {
        unsigned long long mask = __ballot(pred);
        if (mask == 0ull) return;
        int k = __popcll(mask);
        if (n + k > QCAP) drain(cnt_out, out, cap, ctrl);
        if (pred) q[n + static_cast<int>(lane_rank(mask))] = item;
        __builtin_amdgcn_wave_barrier();
        n += k;
    }
};

// Workgroup-wide drain of every wavefront queue with a single global atomic.
// s_fill: LDS int[NW]; s_base: LDS uint32.  Must be called by all threads.
template <int B, int QCAP>
__device__ __forceinline__ void block_drain(WaveQueue<QCAP> &wq, int *s_fill, uint32_t *s_base,
                                            uint32_t *cnt_out, int *out, uint32_t cap, Ctrl *ctrl) {
    constexpr int NW = B / kWave;
    const int wid = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) s_fill[wid] = wq.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) total += static_cast<uint32_t>(s_fill[k]);
        uint32_t base = total ? atomicAdd(cnt_out, total) : 0u;
        if (total && (base + total > cap || base + total < base)) set_error(ctrl, kErrOverflow, false);
        *s_base = base;
    }
    __syncthreads();
    uint32_t base = *s_base;
    for (int k = 0; k < wid; ++k) base += static_cast<uint32_t>(s_fill[k]);
    for (int j = lane_id(); j < wq.n; j += kWave) {
        uint32_t dst = base + static_cast<uint32_t>(j);
        if (dst < cap && dst >= base) out[dst] = wq.q[j];
    }
    wq.n = 0;
}

// ---------------------------------------------------------------------------
// Grid-wide barrier among co-resident workgroups (SyncRunningThreads,
// Section 3.4).  Safe only when every workgroup of the grid is resident at
// once, which the cooperative launch guarantees (or refuses to launch).
//
// Two-level arrival tree.  Workgroup b arrives on the counter of group
// b mod 8; the last arrival of a group arrives on the top counter; the last
// top arrival publishes the new generation.  Counters only grow during a
// launch, so "last" is recognised from the value the fetch_add returns and
// nothing is reset.  Waiters poll only the generation word (a line of its
// own) with s_sleep back-off and relaxed loads.
//
// Coherence.  Each XCD has a private L2, so data written before the barrier
// must be written back from the writer's L2 and stale lines dropped from the
// reader's caches.  Three schemes:
//   kBarWorkgroup: every arrival is an agent-scope acq_rel RMW (an L2
//     write-back and invalidate per workgroup), then an acquire on exit.
//   kBarXcd: the hardware deals workgroups round-robin to the XCDs, so group
//     b mod 8 is exactly one XCD's workgroups and they share one L2.  Every
//     wave first waits until its own stores are acknowledged by that L2
//     (s_waitcnt: __syncthreads alone does not wait for stores), so when a
//     workgroup arrives its stores are in the L2 and ONE write-back by the
//     group's last arrival covers the whole group; every workgroup still
//     takes an acquire (L1 + L2 invalidate) on exit.  (Measured at 1024 workgroups: 9.3 us
//     per barrier against 22.8 us for kBarWorkgroup, no stale reads.  Doing
//     the invalidate once per XCD and dropping only each CU's L1 measured
//     faster but read stale data, so every workgroup keeps its acquire.)
// kBarXcd is correct only under round-robin dispatch, which every workgroup
// checks against the hardware XCC id before its first barrier; the first
// barrier of a launch always uses kBarWorkgroup and, if any workgroup of the
// team found another mapping, the launch stays on kBarWorkgroup.
//
// Every wait gives up when `fatal` is raised or its own wall-clock deadline
// passes (raising `fatal` itself), so every wait ends.  Workgroup 0 reads
// the optional host abort flag before it arrives; the barrier cannot
// complete before that read, so a raised flag is seen by every waiting
// workgroup as `fatal`.  Returns false when the caller must leave the loop.
// ---------------------------------------------------------------------------
constexpr uint32_t kBarXcd = 0;
constexpr uint32_t kBarWorkgroup = 1;

struct BarrierState {
    uint32_t epoch;               // barriers passed by this workgroup
    unsigned long long wd_ticks;  // watchdog in wall-clock ticks
    uint32_t want;                // requested scheme (kBar*)
    uint32_t kind;                // scheme in use (kBarWorkgroup until the mapping is checked)
};

__device__ __forceinline__ BarrierState make_barrier_state(unsigned long long wd_ticks, uint32_t want) {
    return BarrierState{0u, wd_ticks, want, kBarWorkgroup};
}

// Barrier words of a fresh launch (one thread, before the launch that uses them).
__device__ __forceinline__ void reset_barrier_words(Ctrl *c) {
    c->bar_gen = 0;
    c->bar_top = 0;
    for (int g = 0; g < kBarGroups; ++g) {
        c->bar_grp[g].count = 0;
    }
    c->xmap_bad = 0;
}

// The XCD this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ uint32_t xcc_id() {
    return static_cast<uint32_t>(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20)) & 15u;
}


// The workgroups that cooperate on one query: the whole grid of a
// single-query launch, or one group of a batched launch.  Grid-stride loops
// and the barrier use the team, never blockIdx / gridDim directly.
struct Team {
    uint32_t id;    // this workgroup's index in the team
    uint32_t size;  // workgroups in the team
};

__device__ __forceinline__ Team whole_grid() { return Team{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ bool grid_barrier(Ctrl *ctrl, BarrierState &bs, int *s_flag,
                                             const volatile int32_t *abort_flag, Team tm) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        if (bs.epoch == 0 && xcc_id() != blockIdx.x % kBarGroups) atomicOr(&ctrl->xmap_bad, 1u);
        if (abort_flag && tm.id == 0 &&
            __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
            set_error(ctrl, kErrAborted, true);
        const uint32_t G = tm.size;
        const uint32_t ngroups = G < kBarGroups ? G : kBarGroups;
        const uint32_t gid = tm.id % ngroups;
        const uint32_t gsize = G / ngroups + (gid < G % ngroups ? 1u : 0u);
        const uint32_t epoch = ++bs.epoch;
        const bool per_xcd = bs.kind != kBarWorkgroup;
        unsigned long long old;
        if (per_xcd)
            old = __hip_atomic_fetch_add(&ctrl->bar_grp[gid].count, 1ull, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        else
            old = __hip_atomic_fetch_add(&ctrl->bar_grp[gid].count, 1ull, __ATOMIC_ACQ_REL,
                                         __HIP_MEMORY_SCOPE_AGENT);
        const bool last = old + 1 == static_cast<unsigned long long>(epoch) * gsize;
        if (last) {
            unsigned long long top;
            if (per_xcd) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write back this XCD's L2
                top = __hip_atomic_fetch_add(&ctrl->bar_top, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                top = __hip_atomic_fetch_add(&ctrl->bar_top, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (top + 1 == static_cast<unsigned long long>(epoch) * ngroups)
                __hip_atomic_store(&ctrl->bar_gen, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        int ok = 1;
        const unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(&ctrl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (load_agent(&ctrl->fatal)) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > bs.wd_ticks) {
                set_error(ctrl, kErrWatchdog, true);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // after the first barrier every workgroup's mapping check is visible
        if (epoch == 1) bs.kind = load_agent(&ctrl->xmap_bad) ? kBarWorkgroup : bs.want;
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

}  // namespace irgl
