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
    uint32_t t_bitmap;   // bitmap refresh point (new items since the last refresh)
    uint32_t gang;       // server: run on the whole grid (all teams together)
    uint32_t pad;
};

struct BatchParams {
    const TaskDesc *tasks;
    int32_t ntasks;
    uint32_t *queue_head;      // next task to take (one word, reset by the host's init)
    uint32_t *team_task;       // per team: the task it runs (published by its leader)
    char *scratch;             // team t's scratch starts at scratch + t * team_bytes
    unsigned long long team_bytes;
    // offsets inside one team's scratch
    unsigned long long off_wl0, off_wl1, off_stamp, off_shadow, off_far0, off_far1, off_far_flag, off_visited,
        off_hub_v, off_hub_base, off_expd;
    uint32_t cap;              // worklist capacity = largest n
    uint32_t hub_cap;
    int32_t team;              // workgroups per team
    int32_t t_wave, t_block, t_grid;
    unsigned long long wd_ticks;
    uint32_t barrier;  // grid-barrier coherence scheme (kBar*)
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
    p.shadow = sssp ? reinterpret_cast<uint32_t *>(base + bp.off_shadow) : nullptr;
    p.far0 = sssp ? reinterpret_cast<int32_t *>(base + bp.off_far0) : nullptr;
    p.far1 = sssp ? reinterpret_cast<int32_t *>(base + bp.off_far1) : nullptr;
    p.far_flag = sssp ? reinterpret_cast<uint32_t *>(base + bp.off_far_flag) : nullptr;
    p.far_cap = static_cast<uint32_t>(t.n);
    p.expd = sssp ? reinterpret_cast<uint32_t *>(base + bp.off_expd) : nullptr;
    p.split = nullptr;  // batched tasks run on the caller's rows (no light/heavy partition)
    p.hlist = nullptr;
    p.hstamp = nullptr;
    p.hcap = 0;
    p.inv = nullptr;  // results are written under the caller's ids directly
    p.out_caller = nullptr;
    p.parent_caller = nullptr;
    // SSSP without refreshes would only test a bitmap holding the source
    p.visited = (sssp && t.t_bitmap == kInf) ? nullptr : reinterpret_cast<uint32_t *>(base + bp.off_visited);
    p.t_bitmap = t.t_bitmap;
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
    p.src_orig = t.src;
    p.perm = nullptr;  // batched tasks run on the caller's labelling
    p.it = 0;
    p.wd_ticks = bp.wd_ticks;
    p.barrier = bp.barrier;
    p.abort_flag = nullptr;
    p.trace_len = 0;
    p.trace = nullptr;
    p.delta = sssp ? t.delta : kInf;
    p.thresh = p.delta;
    p.far_tr = 0;
    p.refresh = 0;
    p.frontier = nullptr;  // batched BFS runs top-down
    p.frontier2 = nullptr;
    p.do_alpha = 0;
    p.do_beta = 0;
    p.m = 0;
    p.reduce_all = 0;
    p.tail_div = 0;  // without the split the bucketing runs to its end
    p.shadow16 = 0;
    p.pull_heavy_div = 0;
    p.pull_open_div = 0;
    p.step_grow = 0;
    p.heavy_m = 0;
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
    s->heavy_pulls = 0;
    s->frontier_edges = __hip_atomic_load(&p.ctrl->fedges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    add_block_total<B>(r.fedges, &ctrl->fedges);
    // every workgroup's edge count and pushes are in before the leader reads them
    if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) return false;
    if (td.kind == 1 && td.parent) {
        // deterministic SSSP parents: identity worklist over the team
        const int wid = threadIdx.x / kWave;
        Pushers pu{{sm.queue[wid], 0}, {sm.queue_far[wid], 0}, Sink{nullptr, nullptr, 0u, ctrl, nullptr},
                   Sink{nullptr, nullptr, 0u, ctrl, nullptr}, kInf};
        unsigned long long pe = 0;
        const SsspParentOp op{p.val, p.w, p.parent, p.src, p.perm};
        expand<B, SsspParentOp>(nullptr, static_cast<uint32_t>(p.n), static_cast<uint32_t>(p.n), p.row_ptr,
                                p.col, op, sm, pu, p.t_wave, p.t_block, 0, nullptr, nullptr, 0u, nullptr, pe,
                                tm, nullptr);
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
    BarrierState bs = make_barrier_state(bp.wd_ticks, bp.barrier);
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
// next published slot with a CAS on the device head word, copies the
// descriptor to its team's scratch, and the team barrier hands it to the
// team.  When the task is done the leader writes its statistics to the host
// ring, releases the outputs at system scope, and raises the slot's done
// word.
//
// Gangs.  A descriptor marked `gang` (a task on a large graph) runs on the
// WHOLE grid instead, in ring order: its claim sets the pending bit of the
// head word, every team joins it when it next looks for work (after its
// current task), and the grid-wide gang barrier starts it.  The head word
// packs the descriptors claimed (bits 0-31), the gangs started in this
// launch (bits 32-62) and the pending bit (63); a plain claim needs the
// pending bit clear, so no team starts another task while a gang gathers.
// Leaving is a gang too: team 0 posts an exit gang on a host stop request or
// after idle_ticks without work, and after the gang barrier workgroup 0
// decides for the whole grid whether to end (stop, or still no work) or go
// on, so the grid always ends together.  Every wait is bounded (watchdog).
//
// Residency.  The barriers assume every workgroup of the grid is resident.
// A cooperative launch sizes the grid for an otherwise idle device, but a
// kernel on another stream (the caller's own work between requests) can
// still hold part of it while the server's workgroups are dispatched; the
// resident teams would then claim descriptors that can never be run.  So no
// workgroup claims anything before all of them have checked in on the start
// word.  If they are not all in within start_ticks, one CAS decides that the
// launch gives up: every workgroup leaves at once, nothing is claimed, and
// the host launches again while work is pending.  A descriptor claimed by a
// team whose join barrier still fails (watchdog) is reported with the
// watchdog status by its claimer, never left claimed and unreported.
// ---------------------------------------------------------------------------
struct ServerParams {
    BatchParams bp;                 // team layout and thresholds (bp.tasks unused)
    BatchParams gang;               // the gang region's layout (scratch = its base)
    TaskDesc *ring;                 // HOST pinned, ring_cap descriptors
    const uint32_t *tail;           // HOST pinned: descriptors published so far
    unsigned long long *head;       // device: claimed | gangs << 32 | pending << 63
    uint32_t *done;                 // HOST pinned: per slot, (ticket + 1) when finished
    Stats *host_stats;              // HOST pinned: per slot statistics
    const uint32_t *stop;           // HOST pinned: stop request
    uint32_t *start_fails;          // HOST pinned: launches that gave up at the start check
    uint32_t ring_cap;
    unsigned long long idle_ticks;
    unsigned long long start_ticks; // deadline of the start check
};

// What the gang region holds after its control block: the claimed
// descriptor and what the gang is for.
struct GangInfo {
    TaskDesc desc;
    uint32_t ticket;
    uint32_t kind;         // kGangTask or kGangExit
    uint32_t decision;     // exit gang: 1 = end the launch
    uint32_t start_count;  // workgroups checked in at the start of this launch
    uint32_t start_state;  // 0 = checking in, 1 = all resident, 2 = launch gives up
    uint32_t pad;
};
constexpr uint32_t kStartGo = 1;
constexpr uint32_t kStartGiveUp = 2;
constexpr uint32_t kGangTask = 1;
constexpr uint32_t kGangExit = 2;
constexpr unsigned long long kPending = 1ull << 63;

__device__ __forceinline__ uint32_t load_sys(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ unsigned long long load_sys64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void copy_desc(TaskDesc *dst, const TaskDesc *ring_slot) {
    static_assert(sizeof(TaskDesc) % 8 == 0, "descriptor copied in 8-byte words");
    // acquire after the tail was seen, then copy word by word
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(ring_slot);
    unsigned long long *d = reinterpret_cast<unsigned long long *>(dst);
    for (unsigned k = 0; k < sizeof(TaskDesc) / 8; ++k) d[k] = load_sys64(src + k);
}

// Statistics of a finished server task to the host ring, the outputs
// released at system scope, then the slot's done word (one thread).
__device__ __forceinline__ void report_task(const ServerParams &sp, const TaskDesc &td, uint32_t ticket, bool ok) {
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
    hs->heavy_pulls = 0;
    hs->frontier_edges = ds->frontier_edges;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __hip_atomic_store(&sp.done[slot], ticket + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
    BarrierState bs = make_barrier_state(bp.wd_ticks, bp.barrier);
    // the gang region: whole-grid control block and descriptor
    char *gbase = sp.gang.scratch;
    Ctrl *gctrl = reinterpret_cast<Ctrl *>(gbase);
    GangInfo *gi = reinterpret_cast<GangInfo *>(gbase + sizeof(Ctrl));
    BarrierState gbs = make_barrier_state(bp.wd_ticks, bp.barrier);
    const Team grid = whole_grid();
    const bool leader = tm.id == 0 && threadIdx.x == 0;
    constexpr uint32_t kGang = 0xFFFFFFFEu;
    constexpr uint32_t kQuit = 0xFFFFFFFFu;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t joined = 0;         // gangs this team has joined (leader's copy)
    uint32_t gang_claim = kNone;  // leader: ticket of the gang it claimed, until the gang starts
    uint32_t task_claim = kNone;  // leader: ticket of the team task it claimed, until the task starts

    // start check: every workgroup resident before anything is claimed
    if (threadIdx.x == 0) {
        if (atomicAdd(&gi->start_count, 1u) + 1u == gridDim.x) atomicCAS(&gi->start_state, 0u, kStartGo);
        const unsigned long long t0 = wall_clock64();
        uint32_t st;
        while ((st = load_agent(&gi->start_state)) == 0u) {
            if (wall_clock64() - t0 > sp.start_ticks) atomicCAS(&gi->start_state, 0u, kStartGiveUp);
            __builtin_amdgcn_s_sleep(2);
        }
        if (st != kStartGo && blockIdx.x == 0)
            __hip_atomic_store(sp.start_fails, load_sys(sp.start_fails) + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        sm.flag = st == kStartGo ? 1 : 0;
    }
    __syncthreads();
    if (!sm.flag) return;  // uniform: the launch gave up before claiming anything

    for (;;) {
        if (leader) {
            uint32_t action = kGang;
            const unsigned long long t0 = wall_clock64();
            for (;;) {
                const unsigned long long hw = __hip_atomic_load(sp.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t h = static_cast<uint32_t>(hw);
                const uint32_t seq = static_cast<uint32_t>(hw >> 32) & 0x7FFFFFFFu;
                if (hw & kPending) {
                    if (seq > joined) {  // a gang this team has not joined yet
                        joined = seq;
                        break;
                    }
                } else if (h < load_sys(sp.tail)) {
                    const TaskDesc *slot = &sp.ring[h % sp.ring_cap];
                    const bool gang = load_sys(&slot->gang) != 0u;
                    const unsigned long long nw =
                        gang ? (kPending | (static_cast<unsigned long long>(seq + 1) << 32) | (h + 1u))
                             : ((hw & ~0xFFFFFFFFull) | (h + 1u));
                    if (atomicCAS(sp.head, hw, nw) == hw) {
                        if (gang) {
                            copy_desc(&gi->desc, slot);
                            gi->ticket = h;
                            gi->kind = kGangTask;
                            joined = seq + 1;
                            gang_claim = h;
                        } else {
                            copy_desc(mine, slot);
                            action = h;
                            task_claim = h;
                        }
                        break;
                    }
                    continue;
                } else if (team_id == 0 && (load_sys(sp.stop) || wall_clock64() - t0 > sp.idle_ticks)) {
                    const unsigned long long nw = kPending | (static_cast<unsigned long long>(seq + 1) << 32) | h;
                    if (atomicCAS(sp.head, hw, nw) == hw) {
                        gi->kind = kGangExit;
                        joined = seq + 1;
                        break;
                    }
                    continue;
                }
                // every wait ends: a leader that finds neither work nor a gang
                // for a whole watchdog period (team 0 gone) ends its team
                if (wall_clock64() - t0 > bp.wd_ticks) {
                    action = kQuit;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            store_agent(&bp.team_task[team_id], action);
        }
        if (!grid_barrier(ctrl, bs, &sm.flag, nullptr, tm)) {
            // the team cannot run what its leader claimed: report it failed
            if (leader) {
                if (task_claim != kNone) report_task(sp, *mine, task_claim, false);
                if (gang_claim != kNone) report_task(sp, gi->desc, gang_claim, false);
            }
            return;
        }
        task_claim = kNone;  // the team has it: run_task's end reports it
        if (threadIdx.x == 0) s_ticket = load_agent(&bp.team_task[team_id]);
        __syncthreads();
        const uint32_t ticket = s_ticket;
        if (ticket == kQuit) return;  // uniform across the team
        if (ticket == kGang) {
            // every team is here: the gang region's descriptor and kind are visible
            if (!grid_barrier(gctrl, gbs, &sm.flag, nullptr, grid)) {
                if (leader && gang_claim != kNone) report_task(sp, gi->desc, gang_claim, false);
                return;
            }
            gang_claim = kNone;  // started: workgroup 0 reports it
            if (gi->kind == kGangExit) {
                if (grid.id == 0 && threadIdx.x == 0) {
                    const uint32_t h = static_cast<uint32_t>(
                        __hip_atomic_load(sp.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    gi->decision = (load_sys(sp.stop) || h >= load_sys(sp.tail)) ? 1u : 0u;
                }
                if (!grid_barrier(gctrl, gbs, &sm.flag, nullptr, grid)) return;
                // a later gang rewrites the kind and descriptor, never the decision
                const bool end = gi->decision != 0u;
                if (grid.id == 0 && threadIdx.x == 0) atomicAnd(sp.head, ~kPending);
                if (end) return;
                continue;
            }
            const TaskDesc td = gi->desc;
            const uint32_t gticket = gi->ticket;
            LoopResult r;
            const bool ok = run_task<B>(sp.gang, td, gbase, grid, gbs, sm, r);
            if (grid.id == 0 && threadIdx.x == 0) {
                report_task(sp, td, gticket, ok);
                atomicAnd(sp.head, ~kPending);
            }
            if (!ok) return;
            continue;
        }
        const TaskDesc td = *mine;
        LoopResult r;
        const bool ok = run_task<B>(bp, td, base, tm, bs, sm, r);
        if (leader) report_task(sp, td, ticket, ok);
        if (!ok) return;
    }
}

}  // namespace irgl
