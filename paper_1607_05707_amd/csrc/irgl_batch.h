// Batched launch: many BFS/SSSP queries of uneven size in ONE persistent
// cooperative launch, fed from a device-resident task queue.
//
// The grid is split into teams of `team` consecutive workgroups.  A team
// takes the next task with one atomicAdd on the queue head (tasks are sorted
// largest first by the host), runs the same outlined Iterate loop as a
// single-query launch with its own barrier and its own scratch (worklists,
// stamps, far lists, bitmap, grid-tier list), writes the task's statistics,
// and takes the next task until the queue is drained.  Both loop bodies (BFS
// and SSSP) live in this one control kernel, so its workgroup size must be
// one that both bodies support (T_control = T_BFS ∩ T_SSSP, Section 4.3).
#pragma once

#include "irgl_query.h"

namespace irgl {

// One task of the table (device copy written by the host).
struct TaskDesc {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    uint32_t *out;
    int32_t *parent;
    Stats *stats;        // per-task statistics (device)
    int32_t n;
    int32_t kind;        // 0 BFS, 1 SSSP
    int32_t src;
    uint32_t delta;
    uint32_t max_iter;
    uint32_t pad;
};

// Per-team scratch, carved from the batch workspace (sizes for the largest
// task of the batch).
struct TeamScratch {
    Ctrl *ctrl;
    int32_t *wl0, *wl1;
    uint32_t *stamp;
    int32_t *far0, *far1;
    uint32_t *far_flag;
    uint32_t *visited;
    int32_t *hub_v;
    uint32_t *hub_base;
};

struct BatchParams {
    const TaskDesc *tasks;
    int32_t ntasks;
    uint32_t *queue_head;      // next task to take (one word, reset by the host's init)
    uint32_t *team_task;       // per team: the task it runs (published by its leader)
    char *scratch;             // team t's scratch starts at scratch + t * team_bytes
    unsigned long long team_bytes;
    // offsets inside one team's scratch
    unsigned long long off_wl0, off_wl1, off_stamp, off_far0, off_far1, off_far_flag, off_visited,
        off_hub_v, off_hub_base;
    uint32_t cap;              // worklist capacity = largest n
    uint32_t hub_cap;
    int32_t team;              // workgroups per team
    int32_t t_wave, t_block, t_grid;
    uint32_t t_bitmap_div;     // refresh the bitmap when frontier >= n / t_bitmap_div
    unsigned long long wd_ticks;
};

__device__ __forceinline__ Params task_params(const BatchParams &bp, const TaskDesc &t, char *base) {
    Params p;
    p.n = t.n;
    p.row_ptr = t.row_ptr;
    p.col = t.col;
    p.w = t.w;
    p.val = t.out;
    p.parent = t.parent;
    p.ctrl = reinterpret_cast<Ctrl *>(base);
    p.wl0 = reinterpret_cast<int32_t *>(base + bp.off_wl0);
    p.wl1 = reinterpret_cast<int32_t *>(base + bp.off_wl1);
    const bool sssp = t.kind == 1;
    p.stamp = sssp ? reinterpret_cast<uint32_t *>(base + bp.off_stamp) : nullptr;
    p.far0 = sssp ? reinterpret_cast<int32_t *>(base + bp.off_far0) : nullptr;
    p.far1 = sssp ? reinterpret_cast<int32_t *>(base + bp.off_far1) : nullptr;
    p.far_flag = sssp ? reinterpret_cast<uint32_t *>(base + bp.off_far_flag) : nullptr;
    p.far_cap = static_cast<uint32_t>(t.n);
    p.visited = sssp ? nullptr : reinterpret_cast<uint32_t *>(base + bp.off_visited);
    p.t_bitmap = max(1u, static_cast<uint32_t>(t.n) / bp.t_bitmap_div);
    p.hub_v = reinterpret_cast<int32_t *>(base + bp.off_hub_v);
    p.hub_base = reinterpret_cast<uint32_t *>(base + bp.off_hub_base);
    p.hub_cap = bp.hub_cap;
    p.dstats = t.stats;
    p.cap = min(bp.cap, static_cast<uint32_t>(t.n));
    p.max_iter = t.max_iter;
    p.t_wave = bp.t_wave;
    p.t_block = bp.t_block;
    p.t_grid = bp.t_grid;
    p.src = t.src;
    p.it = 0;
    p.wd_ticks = bp.wd_ticks;
    p.abort_flag = nullptr;
    p.trace_len = 0;
    p.trace = nullptr;
    p.delta = sssp ? t.delta : kInf;
    p.thresh = p.delta;
    p.far_tr = 0;
    return p;
}

// Statistics of a finished task, written by the team leader after the
// team's last barrier of the task.
__device__ __forceinline__ void write_task_stats(const Params &p, const LoopResult &r, Team tm, int block) {
    Stats *s = p.dstats;
    if (!s) return;
    s->status = static_cast<int32_t>(load_agent(&p.ctrl->error));
    s->iterations = r.iterations;
    s->items = r.items;
    s->edges = __hip_atomic_load(&p.ctrl->edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s->max_frontier = r.max_frontier;
    s->grid = static_cast<int32_t>(tm.size);
    s->block = block;
    s->reserved = 0;
}

// Run one task on a team: fill, Iterate loop, optional SSSP parent pass.
// All threads of the team call it; returns false when the team must stop
// (a fatal error: watchdog).  On return every workgroup has passed the
// team's last barrier of the task, and the leader has the statistics.
template <int B>
__device__ __forceinline__ bool run_task(const BatchParams &bp, const TaskDesc &td, char *base, Team tm,
                                         BarrierState &bs, Smem<B> &sm, LoopResult &r) {
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(base);
    const bool leader = tm.id == 0 && threadIdx.x == 0;
    const Params p = task_params(bp, td, base);
    init_arrays(p, td.kind == 1 ? 1 : 0, tm);
    if (leader) init_control(p, false);
    if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return false;
    if (td.kind == 1) r = run_iterate<B, SsspOp>(p, sm, tm, bs);
    else r = run_iterate<B, BfsOp>(p, sm, tm, bs);
    add_block_total<B>(r.edges, &ctrl->edges);
    // every workgroup's edge count and pushes are in before the leader reads them
    if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return false;
    if (td.kind == 1 && td.parent) {
        // deterministic SSSP parents: identity worklist over the team
        const int wid = threadIdx.x / kWave;
        Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{nullptr, nullptr, 0u, ctrl, nullptr},
                   Sink{nullptr, nullptr, 0u, ctrl, nullptr}, kInf};
        unsigned long long pe = 0;
        const SsspParentOp op{p.val, p.w, p.parent, p.src};
        expand<B, SsspParentOp>(nullptr, static_cast<uint32_t>(p.n), static_cast<uint32_t>(p.n), p.row_ptr,
                                p.col, op, sm, pu, p.t_wave, p.t_block, 0, nullptr, nullptr, 0u, nullptr, pe,
                                tm);
        if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return false;
    }
    if (leader) write_task_stats(p, r, tm, B);
    return load_agent(&ctrl->fatal) == 0u;  // uniform: set before the last barrier
}

template <int B>
__global__ __launch_bounds__(B) void batch_kernel(BatchParams bp) {
    __shared__ Smem<B> sm;
    __shared__ int s_task;
    const uint32_t team_id = blockIdx.x / static_cast<uint32_t>(bp.team);
    const Team tm{blockIdx.x % static_cast<uint32_t>(bp.team), static_cast<uint32_t>(bp.team)};
    char *base = bp.scratch + static_cast<unsigned long long>(team_id) * bp.team_bytes;
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(base);
    BarrierState bs{0u, bp.wd_ticks};
    const bool leader = tm.id == 0 && threadIdx.x == 0;

    for (;;) {
        // the leader takes the next task and publishes it to the team
        if (leader) {
            const uint32_t t = atomicAdd(bp.queue_head, 1u);
            store_agent(&bp.team_task[team_id], t);
        }
        if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return;
        if (threadIdx.x == 0) s_task = static_cast<int>(load_agent(&bp.team_task[team_id]));
        __syncthreads();
        const int t = s_task;
        if (t >= bp.ntasks) return;  // uniform across the team: queue drained
        LoopResult r;
        if (!run_task<B>(bp, bp.tasks[t], base, tm, bs, sm, r)) return;
    }
}

// ---------------------------------------------------------------------------
// Server: the same teams, fed from a ring of task descriptors in host pinned
// memory while the kernel runs (continuous batching).  The host writes a
// descriptor, then publishes it by raising *tail.  A team leader claims the
// next published slot with a CAS on the device head counter, copies the
// descriptor to its team's scratch, and the team barrier hands it to the
// team.  When the task is done the leader writes its statistics to the host
// ring, releases the outputs at system scope, and raises the slot's done
// word.  A leader that finds no work polls with back-off and ends its team
// when the host raises *stop or after idle_ticks without a task (every wait
// is bounded).
// ---------------------------------------------------------------------------
struct ServerParams {
    BatchParams bp;                 // team layout and thresholds (bp.tasks unused)
    TaskDesc *ring;                 // HOST pinned, ring_cap descriptors
    const uint32_t *tail;           // HOST pinned: descriptors published so far
    uint32_t *head;                 // device: descriptors claimed so far
    uint32_t *done;                 // HOST pinned: per slot, (ticket + 1) when finished
    Stats *host_stats;              // HOST pinned: per slot statistics
    const uint32_t *stop;           // HOST pinned: stop request
    uint32_t ring_cap;
    unsigned long long idle_ticks;
};

__device__ __forceinline__ uint32_t load_sys(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ unsigned long long load_sys64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int B>
__global__ __launch_bounds__(B) void server_kernel(ServerParams sp) {
    __shared__ Smem<B> sm;
    __shared__ uint32_t s_ticket;
    const BatchParams &bp = sp.bp;
    const uint32_t team_id = blockIdx.x / static_cast<uint32_t>(bp.team);
    const Team tm{blockIdx.x % static_cast<uint32_t>(bp.team), static_cast<uint32_t>(bp.team)};
    char *base = bp.scratch + static_cast<unsigned long long>(team_id) * bp.team_bytes;
    Ctrl *ctrl = reinterpret_cast<Ctrl *>(base);
    // this team's copy of the claimed descriptor (right after the control block)
    TaskDesc *mine = reinterpret_cast<TaskDesc *>(base + sizeof(Ctrl));
    static_assert(sizeof(TaskDesc) % 8 == 0, "descriptor copied in 8-byte words");
    BarrierState bs{0u, bp.wd_ticks};
    const bool leader = tm.id == 0 && threadIdx.x == 0;
    constexpr uint32_t kNone = 0xFFFFFFFFu;

    for (;;) {
        if (leader) {
            uint32_t claimed = kNone;
            const unsigned long long t0 = wall_clock64();
            for (;;) {
                const uint32_t h = load_agent(sp.head);
                const uint32_t tl = load_sys(sp.tail);
                if (h < tl) {
                    if (atomicCAS(sp.head, h, h + 1) == h) {
                        claimed = h;
                        break;
                    }
                    continue;
                }
                if (load_sys(sp.stop) || wall_clock64() - t0 > sp.idle_ticks) break;
                __builtin_amdgcn_s_sleep(8);
            }
            if (claimed != kNone) {
                // descriptor: acquire after the tail was seen, then copy word by word
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                const unsigned long long *src = reinterpret_cast<const unsigned long long *>(
                    &sp.ring[claimed % sp.ring_cap]);
                unsigned long long *dst = reinterpret_cast<unsigned long long *>(mine);
                for (unsigned k = 0; k < sizeof(TaskDesc) / 8; ++k) dst[k] = load_sys64(src + k);
            }
            store_agent(&bp.team_task[team_id], claimed);
        }
        if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return;
        if (threadIdx.x == 0) s_ticket = load_agent(&bp.team_task[team_id]);
        __syncthreads();
        const uint32_t ticket = s_ticket;
        if (ticket == kNone) return;  // uniform across the team
        const TaskDesc td = *mine;
        LoopResult r;
        const bool ok = run_task<B>(bp, td, base, tm, bs, sm, r);
        if (leader) {
            // statistics to the host ring, outputs released at system scope, then the done word
            const uint32_t slot = ticket % sp.ring_cap;
            Stats *hs = &sp.host_stats[slot];
            const Stats *ds = td.stats;
            hs->status = ok ? ds->status : static_cast<int32_t>(kErrWatchdog);
            hs->iterations = ds->iterations;
            hs->items = ds->items;
            hs->edges = ds->edges;
            hs->max_frontier = ds->max_frontier;
            hs->grid = ds->grid;
            hs->block = ds->block;
            hs->reserved = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            __hip_atomic_store(&sp.done[slot], ticket + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        if (!ok) return;
    }
}

}  // namespace irgl
