// Outlined pipes (Section 4.2, Compiling Pipe; Section 4.3, Compiling Kernel
// Invocations): a host-built program of orchestration statements (Invoke,
// Iterate, Pipe / Pipe Once, run-time choice of the next kernel) runs in ONE
// cooperative persistent launch.  The control kernel interprets the program;
// every workgroup executes the same statements with the same uniform state,
// since every decision reads counters that a grid barrier has settled.  A
// kernel invocation is a device-function call followed by a grid barrier.
//
// Pipe context.  Three worklist buffers play the roles in / out / retry.  An
// invocation pops `in` and pushes `out` and `retry`; the counts it produces
// live in rotating counters indexed by the invocation number.  Invocation i
// pushes through cnt[i % 3], which every workgroup reads right after the
// barrier that ends i, and clears cnt[(i + 1) % 3] for the next invocation:
// that counter was last read after the barrier ending i - 2, before each
// workgroup arrived at the barrier ending i - 1.  (Clearing cnt[(i + 2) % 3]
// would let a workgroup that starts invocation i + 1 early clear the count
// of i while a slower workgroup has yet to read it.)  Every workgroup keeps
// the roles and the counts of the context in registers:
//   - after a body that uses worklists: in <-> out, |in| = |out|;
//   - after a body that uses `retry` with a non-empty retry list: in <-> retry
//     and the body runs again; `out` keeps filling (its base offset grows);
//   - a body without worklists leaves the context as it is.
//
// T_control.  Each body declares its class (ElasticBlock, ShrinkableBlock,
// FixedBlock) and its LDS layout; the host intersects the sets of workgroup
// sizes they admit and launches the control kernel instantiated for the
// largest common size.  A body is compiled into the control kernel only for
// the sizes its class admits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "irgl.h"
#include "irgl_expand.h"

namespace irgl_shared {
irgl_status note_hip_failure(hipError_t e);
irgl_status caller_csr(const irgl_graph_s *g, int *device, irgl_csr *out);
}  // namespace irgl_shared

namespace irgl {
namespace pipe {

constexpr int kDepth = 8;                  // deepest BEGIN nesting
constexpr unsigned long long kNoKey = ~0ull;
constexpr int kInitBlock = 256;            // MST_INIT's compaction layout is built for this size
constexpr int kPullFraction = 16;          // IRGL_COND_FRONTIER_LARGE: |in| >= n / 16

struct BodyInfo {
    bool uses_wl;     // pops `in` and/or pushes `out`
    bool uses_retry;  // pushes `retry`
    bool reduces;     // returns Any(...) through ReduceAndReturn
    bool bfs;         // advances the BFS level
    bool mst;         // needs the Boruvka state
    int kind;         // IRGL_BLOCK_*
    int block;
};

// Traits of every body (host and device).
__host__ __device__ inline BodyInfo body_info(int b) {
    switch (b) {
        case IRGL_BODY_BFS_PUSH: return {true, false, false, true, false, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_BFS_PULL: return {true, false, false, true, false, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_MST_INIT: return {true, false, false, false, true, IRGL_BLOCK_FIXED, kInitBlock};
        case IRGL_BODY_MST_FINDMIN: return {true, true, false, false, true, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_MST_HOOK: return {false, false, false, false, true, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_MST_JUMP: return {false, false, true, false, true, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_MST_RELABEL: return {false, false, false, false, true, IRGL_BLOCK_ELASTIC, 1024};
        case IRGL_BODY_MST_MINID: return {false, false, false, false, true, IRGL_BLOCK_ELASTIC, 1024};
        default: return {false, false, false, false, true, IRGL_BLOCK_ELASTIC, 1024};  // MST_LABEL
    }
}

// LDS of the bodies.  BFS_PUSH runs the nested edge scheduler (Smem<B>: a
// per-thread gather window and per-wavefront push queues); the other
// worklist bodies stage pushes in per-wavefront queues (out and retry);
// MST_INIT compacts with a workgroup scan laid out for kInitBlock threads.
template <int B>
struct QueueSmem {
    int q_out[B / kWave][kQueueCap];
    int q_retry[B / kWave][kQueueCap];
    int fill[B / kWave];
    uint32_t base;
};
struct InitSmem {
    int wsum[kInitBlock / kWave];
    uint32_t base;
};
template <int B>
union PipeSmem {
    Smem<B> nested;
    QueueSmem<B> queues;
    InitSmem init;
};

template <int B>
constexpr size_t body_lds(int b) {
    return b == IRGL_BODY_BFS_PUSH ? sizeof(Smem<B>)
         : b == IRGL_BODY_MST_INIT ? sizeof(InitSmem)
         : body_info(b).uses_wl ? sizeof(QueueSmem<B>) : 0;
}

struct Counters {  // one 128-byte line
    uint32_t out[3];
    uint32_t retry[3];
    uint32_t red[3];
    uint32_t pad[23];
};
static_assert(sizeof(Counters) == 128, "pipe counters");

struct Params {
    int32_t n;
    long long m;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    const irgl_pipe_op *prog;
    int32_t nops;
    int32_t src;
    Ctrl *ctrl;
    Counters *cnt;
    int32_t *wl[3];
    uint32_t cap;
    uint32_t *level;
    // Boruvka state
    int32_t *comp;               // component (root id) of every vertex
    int32_t *hookto;             // per root: the root it joins this round, or -1
    int32_t *minv;               // per root: smallest vertex id of its tree
    unsigned long long *cmin;    // per root: candidate key (weight << 32 | canonical entry)
    int32_t *cfar;               // ... the root at the candidate's other end
    int32_t *crev;               // ... and the candidate's other CSR entry
    uint32_t *lock;              // per root: lock word of the atomic section
    int32_t *component;
    uint8_t *in_forest;
    unsigned long long *weight;
    int32_t *trace;
    uint32_t trace_len;
    uint32_t max_inv;
    unsigned long long wd_ticks;
    uint32_t barrier;
    uint32_t force_retry;
    Stats *dstats;
};

// The uniform state every workgroup keeps while it interprets the program.
struct State {
    int in_b, out_b, retry_b;   // buffer of each role
    uint32_t in_n;              // items in `in`
    uint32_t out_base;          // items already in `out` from earlier retry rounds
    uint32_t inv;               // invocations so far
    uint32_t level;             // BFS: level of the current frontier
    bool any;                   // last ReduceAndReturn result
    unsigned long long items, edges;
    uint32_t max_in;
    uint32_t round;             // retry round of the current invocation (0: first)
};

// ---------------------------------------------------------------------------
// Bodies.  Every thread of every workgroup calls a body; pushes go through
// the wavefront queues (one atomic per queue drain, one per workgroup at the
// end), which the caller drains.
// ---------------------------------------------------------------------------

// Top-down BFS level: the library's nested edge scheduler and check-and-label
// operator on `in` (no grid tier: a body is one phase between two barriers).
template <int B>
__device__ void bfs_push(const Params &p, PipeSmem<B> &sm, Team tm, State &s, Pushers &pu) {
    const BfsOp op{p.level, nullptr, nullptr, s.level + 1, nullptr};
    unsigned long long edges = 0;
    expand<B, BfsOp>(p.wl[s.in_b], s.in_n, static_cast<uint32_t>(p.n), p.row_ptr, p.col, op, sm.nested, pu, 2 * B,
                     2 * B, 0, nullptr, nullptr, 0u, nullptr, edges, tm, nullptr);
    s.edges += edges;
}

// Bottom-up BFS level: every unvisited vertex looks for a neighbour labelled
// with the current level; the thread that owns the vertex labels it (plain
// store: no other writer) and pushes it.
template <int B>
__device__ void bfs_pull(const Params &p, Team tm, State &s, Pushers &pu) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    const uint32_t cur = s.level;
    unsigned long long edges = 0;
    for (uint32_t base = tm.id * B; base < n; base += tm.size * B) {
        const uint32_t v = base + threadIdx.x;
        bool found = false;
        if (v < n && p.level[v] == kInf) {
            const int r1 = p.row_ptr[v + 1];
            for (int e = p.row_ptr[v]; e < r1; ++e) {
                ++edges;
                if (p.level[p.col[e]] == cur) {
                    found = true;
                    break;
                }
            }
            if (found) p.level[v] = cur + 1;
        }
        pu.near(found, static_cast<int>(v));
    }
    s.edges += edges;
}

// Boruvka state reset and the initial worklist: every vertex with an edge.
// The workgroup compacts its tile of kInitBlock vertices with a scan laid
// out for exactly that size and appends it with one atomic.
template <int B>
__device__ void mst_init(const Params &p, PipeSmem<B> &sm, Team tm, State &s) {
    if constexpr (B == kInitBlock) {
        const uint32_t n = static_cast<uint32_t>(p.n);
        const unsigned long long m = static_cast<unsigned long long>(p.m);
        const unsigned long long big = m > n ? m : n;
        for (unsigned long long i = tm.id * B + threadIdx.x; i < big; i += static_cast<unsigned long long>(tm.size) * B) {
            if (i < n) {
                p.comp[i] = static_cast<int32_t>(i);
                p.hookto[i] = -1;
                p.minv[i] = INT_MAX;
                p.cmin[i] = kNoKey;
                p.lock[i] = 0u;
            }
            if (i < m) p.in_forest[i] = 0;
        }
        if (tm.id == 0 && threadIdx.x == 0) *p.weight = 0ull;
        const int lane = lane_id(), wid = threadIdx.x / kWave;
        int32_t *out = p.wl[s.out_b];
        for (uint32_t base = tm.id * B; base < n; base += tm.size * B) {
            const uint32_t v = base + threadIdx.x;
            const int flag = (v < n && p.row_ptr[v + 1] > p.row_ptr[v]) ? 1 : 0;
            const int incl = wave_inclusive_scan(flag);
            if (lane == kWave - 1) sm.init.wsum[wid] = incl;
            __syncthreads();
            int pre = 0, total = 0;
#pragma unroll
            for (int k = 0; k < kInitBlock / kWave; ++k) {
                pre += k < wid ? sm.init.wsum[k] : 0;
                total += sm.init.wsum[k];
            }
            if (threadIdx.x == 0) sm.init.base = total ? atomicAdd(&p.cnt->out[s.inv % 3], static_cast<uint32_t>(total)) : 0u;
            __syncthreads();
            const uint32_t slot = sm.init.base + static_cast<uint32_t>(pre + incl - flag);
            if (flag && slot < p.cap) out[slot] = static_cast<int32_t>(v);
            __syncthreads();  // wsum and base are rewritten by the next tile
        }
    } else {
        // not reachable: the host launches no size outside this body's set
        if (threadIdx.x == 0) set_error(p.ctrl, kErrInternal, true);
    }
}

// Index of the u -> v entry of row u (rows sorted by destination), or -1.
__device__ __forceinline__ int32_t find_entry(const Params &p, int32_t u, int32_t v) {
    int lo = p.row_ptr[u], hi = p.row_ptr[u + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (p.col[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return (lo < p.row_ptr[u + 1] && p.col[lo] == v) ? lo : -1;
}

// Find-min-edge with a non-blocking atomic section.  For each popped vertex:
// its lightest edge to another component, in the order (weight, smaller
// endpoint, larger endpoint).  A candidate that cannot beat the component's
// current one (weights only fall in this phase, so a stale read is only
// larger) is done; otherwise the lane tries the component's lock ONCE:
// holding it, it re-checks and writes the candidate's three words together
// (key, the other root, the reverse entry); the lock busy, the vertex goes
// to `retry` (Atomic ... Else).  A vertex that had a cross edge is pushed
// to `out` for the next round.
template <int B>
__device__ void mst_findmin(const Params &p, Team tm, State &s, Pushers &pu, Pushers &pr) {
    const int32_t *in = p.wl[s.in_b];
    unsigned long long edges = 0;
    for (uint32_t base = tm.id * B; base < s.in_n; base += tm.size * B) {
        const uint32_t i = base + threadIdx.x;
        bool to_out = false, to_retry = false;
        int32_t v = 0;
        if (i < s.in_n) {
            v = in[i];
            const int32_t c = p.comp[v];
            uint32_t bw = kInf;
            int32_t ba = INT_MAX, bb = INT_MAX, be = -1;
            const int r1 = p.row_ptr[v + 1];
            for (int e = p.row_ptr[v]; e < r1; ++e) {
                ++edges;
                const int32_t d = p.col[e];
                if (d == v || p.comp[d] == c) continue;
                const uint32_t wt = p.w[e];
                const int32_t a = v < d ? v : d, b = v < d ? d : v;
                if (wt < bw || (wt == bw && (a < ba || (a == ba && b < bb)))) {
                    bw = wt;
                    ba = a;
                    bb = b;
                    be = e;
                }
            }
            if (be >= 0) {
                const int32_t d = p.col[be];
                const int32_t back = find_entry(p, d, v);     // the d -> v entry
                const int32_t canon = v < d ? be : back;      // the entry from the smaller endpoint
                const int32_t rev = v < d ? back : be;        // ... and the other one
                if (back < 0) {
                    set_error(p.ctrl, kErrInternal, false);  // an edge without its reverse entry
                } else {
                    const unsigned long long key = (static_cast<unsigned long long>(bw) << 32) |
                                                   static_cast<uint32_t>(canon);
                    to_out = true;
                    if (p.force_retry && s.round == 0 && (v & 1)) {
                        to_out = false;  // host-forced Else branch
                        to_retry = true;
                    } else if (key < p.cmin[c]) {
                        unsigned int expect = 0u;
                        if (__hip_atomic_compare_exchange_strong(&p.lock[c], &expect, 1u, __ATOMIC_ACQUIRE,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            const unsigned long long cur = __hip_atomic_load(&p.cmin[c], __ATOMIC_RELAXED,
                                                                             __HIP_MEMORY_SCOPE_AGENT);
                            if (key < cur) {
                                __hip_atomic_store(&p.cmin[c], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_store(&p.cfar[c], p.comp[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_store(&p.crev[c], rev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
                            __hip_atomic_store(&p.lock[c], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            to_out = false;
                            to_retry = true;
                        }
                    }
                }
            }
        }
        pu.near(to_out, v);
        pr.near(to_retry, v);
    }
    s.edges += edges;
}

// Every root with a candidate hooks to the root at the candidate's other
// end, unless the two chose the same edge and this root has the smaller id
// (then it stays a root); the hooking root adds the edge to the forest, so
// every forest edge is added once.
template <int B>
__device__ void mst_hook(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    unsigned long long wsum = 0;
    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B) {
        if (p.comp[v] != static_cast<int32_t>(v)) continue;
        const unsigned long long k = p.cmin[v];
        int32_t h = -1;
        if (k != kNoKey) {
            const int32_t o = p.cfar[v];
            const bool mutual = p.cmin[o] == k;
            if (!mutual || static_cast<int32_t>(v) > o) {
                h = o;
                p.in_forest[static_cast<uint32_t>(k)] = 1;
                p.in_forest[p.crev[v]] = 1;
                wsum += k >> 32;
            }
        }
        p.hookto[v] = h;
    }
    for (int d = 1; d < kWave; d <<= 1) wsum += __shfl_xor(wsum, d, kWave);
    if (lane_id() == 0 && wsum) atomicAdd(p.weight, wsum);
}

// One step of pointer jumping over the hooks of the roots (racing readers see
// an old or a new target, both ancestors); resets the candidates for the
// next round.  Returns whether some hook moved.
template <int B>
__device__ bool mst_jump(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    bool changed = false;
    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B) {
        p.cmin[v] = kNoKey;
        if (p.comp[v] != static_cast<int32_t>(v)) continue;
        const int32_t h = p.hookto[v];
        if (h < 0) continue;
        const int32_t hh = p.hookto[h];
        if (hh >= 0 && hh != h) {
            p.hookto[v] = hh;
            changed = true;
        }
    }
    return changed;
}

template <int B>
__device__ void mst_relabel(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B) {
        const int32_t c = p.comp[v];
        const int32_t h = p.hookto[c];
        if (h >= 0) p.comp[v] = h;
    }
}

template <int B>
__device__ void mst_minid(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B) atomicMin(&p.minv[p.comp[v]], static_cast<int32_t>(v));
}

template <int B>
__device__ void mst_label(const Params &p, Team tm) {
    const uint32_t n = static_cast<uint32_t>(p.n);
    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B) p.component[v] = p.minv[p.comp[v]];
}

// ---------------------------------------------------------------------------
// One invocation of `body` (with its retry rounds): body, drains, barrier,
// then the context update.  Returns false when the launch must stop.
// ---------------------------------------------------------------------------
template <int B>
__device__ bool invoke(const Params &p, PipeSmem<B> &sm, int *s_flag, Team tm, BarrierState &bs, State &s,
                       int body) {
    const BodyInfo bi = body_info(body);
    const bool lead = tm.id == 0 && threadIdx.x == 0;
    for (s.round = 0;; ++s.round) {
        if (s.inv >= p.max_inv) {
            if (lead) set_error(p.ctrl, kErrIterLimit, true);
            return false;
        }
        const uint32_t i = s.inv;
        if (lead) {
            store_agent(&p.cnt->out[(i + 1) % 3], 0u);
            store_agent(&p.cnt->retry[(i + 1) % 3], 0u);
            store_agent(&p.cnt->red[(i + 1) % 3], 0u);
            if (i < p.trace_len) p.trace[i] = body;
        }
        if (bi.uses_wl) {
            s.items += s.in_n;
            s.max_in = max(s.max_in, s.in_n);
        }
        const int wid = threadIdx.x / kWave;
        // pushes to `out` land after the items earlier retry rounds left there
        Pushers pu{{sm.queues.q_out[wid], 0}, {nullptr, 0},
                   Sink{&p.cnt->out[i % 3], p.wl[s.out_b] + s.out_base, p.cap - s.out_base, p.ctrl, nullptr},
                   Sink{}, kInf};
        Pushers pr{{sm.queues.q_retry[wid], 0}, {nullptr, 0},
                   Sink{&p.cnt->retry[i % 3], p.wl[s.retry_b], p.cap, p.ctrl, nullptr}, Sink{}, kInf};
        bool any = false;
        switch (body) {
            case IRGL_BODY_BFS_PUSH:
                pu.nq.q = sm.nested.queue[wid];
                bfs_push<B>(p, sm, tm, s, pu);
                block_drain<B, kQueueCap>(pu.nq, sm.nested.fill, &sm.nested.base, pu.sk.cnt_out, pu.sk.out,
                                          pu.sk.cap, pu.sk.ctrl);
                break;
            case IRGL_BODY_BFS_PULL:
                bfs_pull<B>(p, tm, s, pu);
                block_drain<B, kQueueCap>(pu.nq, sm.queues.fill, &sm.queues.base, pu.sk.cnt_out, pu.sk.out,
                                          pu.sk.cap, pu.sk.ctrl);
                break;
            case IRGL_BODY_MST_INIT: mst_init<B>(p, sm, tm, s); break;
            case IRGL_BODY_MST_FINDMIN:
                mst_findmin<B>(p, tm, s, pu, pr);
                block_drain<B, kQueueCap>(pu.nq, sm.queues.fill, &sm.queues.base, pu.sk.cnt_out, pu.sk.out,
                                          pu.sk.cap, pu.sk.ctrl);
                block_drain<B, kQueueCap>(pr.nq, sm.queues.fill, &sm.queues.base, pr.sk.cnt_out, pr.sk.out,
                                          pr.sk.cap, pr.sk.ctrl);
                break;
            case IRGL_BODY_MST_HOOK: mst_hook<B>(p, tm); break;
            case IRGL_BODY_MST_JUMP: any = mst_jump<B>(p, tm); break;
            case IRGL_BODY_MST_RELABEL: mst_relabel<B>(p, tm); break;
            case IRGL_BODY_MST_MINID: mst_minid<B>(p, tm); break;
            default: mst_label<B>(p, tm); break;
        }
        // ReduceAndReturn: one atomicOr per workgroup, read after the barrier
        if (bi.reduces && __syncthreads_or(any) && threadIdx.x == 0) atomicOr(&p.cnt->red[i % 3], 1u);
        if (!grid_barrier(p.ctrl, bs, s_flag, nullptr, tm)) return false;
        s.inv = i + 1;
        if (bi.bfs) ++s.level;
        if (bi.reduces) s.any = load_agent(&p.cnt->red[i % 3]) != 0u;
        if (!bi.uses_wl) return true;
        const uint32_t o = min(load_agent(&p.cnt->out[i % 3]), p.cap - s.out_base);
        const uint32_t r = bi.uses_retry ? min(load_agent(&p.cnt->retry[i % 3]), p.cap) : 0u;
        if (r > 0) {
            // retry round: in <-> retry, `out` keeps its items
            const int t = s.in_b;
            s.in_b = s.retry_b;
            s.retry_b = t;
            s.in_n = r;
            s.out_base += o;
            continue;
        }
        const int t = s.in_b;
        s.in_b = s.out_b;
        s.out_b = t;
        s.in_n = s.out_base + o;
        s.out_base = 0;
        return true;
    }
}

__device__ __forceinline__ bool condition(const Params &p, const State &s, int c) {
    bool v;
    switch (c & 0xFF) {
        case IRGL_COND_IN_EMPTY: v = s.in_n == 0; break;
        case IRGL_COND_FRONTIER_LARGE:
            v = static_cast<unsigned long long>(s.in_n) * kPullFraction >= static_cast<unsigned long long>(p.n);
            break;
        default: v = s.any; break;
    }
    return (c & IRGL_COND_NOT) ? !v : v;
}

template <int B>
__global__ __launch_bounds__(B) void pipe_kernel(Params p) {
    __shared__ PipeSmem<B> sm;
    __shared__ int s_flag;
    const Team tm = whole_grid();
    BarrierState bs = make_barrier_state(p.wd_ticks, p.barrier);
    State s{0, 1, 2, 0u, 0u, 0u, 0u, false, 0ull, 0ull, 0u, 0u};
    int stack[kDepth];
    int sp = 0;
    int pc = 0;
    bool ok = true;
    // steps of the interpreter are bounded too: every loop of a checked
    // program invokes a body, and invocations are capped
    unsigned long long steps = 0;
    const unsigned long long max_steps = (static_cast<unsigned long long>(p.max_inv) + 2) * (p.nops + 1);
    const bool lead = tm.id == 0 && threadIdx.x == 0;
    while (ok && pc < p.nops) {
        if (++steps > max_steps) {
            if (lead) set_error(p.ctrl, kErrIterLimit, true);
            break;
        }
        const irgl_pipe_op op = p.prog[pc];
        switch (op.op) {
            case IRGL_PIPE_INVOKE:
                ok = invoke<B>(p, sm, &s_flag, tm, bs, s, op.a);
                ++pc;
                break;
            case IRGL_PIPE_ITERATE: {
                const BodyInfo bi = body_info(op.a);
                do {
                    ok = invoke<B>(p, sm, &s_flag, tm, bs, s, op.a);
                } while (ok && (bi.uses_wl ? s.in_n > 0 : s.any));
                ++pc;
                break;
            }
            case IRGL_PIPE_BEGIN:
                stack[sp++] = pc;
                ++pc;
                break;
            case IRGL_PIPE_END: {
                const int begin = stack[sp - 1];
                if (p.prog[begin].a == 0 && s.in_n > 0) {
                    pc = begin + 1;  // a looping Pipe runs again while `in` has items
                } else {
                    --sp;
                    ++pc;
                }
                break;
            }
            case IRGL_PIPE_IF: pc = condition(p, s, op.a) ? pc + 1 : op.b; break;
            case IRGL_PIPE_JUMP: pc = op.a; break;
            default: {  // IRGL_PIPE_INIT_SOURCE
                const uint32_t n = static_cast<uint32_t>(p.n);
                if (p.level)
                    for (uint32_t v = tm.id * B + threadIdx.x; v < n; v += tm.size * B)
                        p.level[v] = static_cast<int32_t>(v) == p.src ? 0u : kInf;
                if (lead) p.wl[s.in_b][0] = p.src;
                s.in_n = 1;
                s.level = 0;
                ok = grid_barrier(p.ctrl, bs, &s_flag, nullptr, tm);
                ++pc;
                break;
            }
        }
    }
    // statistics: per-workgroup counts summed; the last workgroup publishes
    __shared__ unsigned long long s_edges;
    if (threadIdx.x == 0) s_edges = 0;
    __syncthreads();
    atomicAdd(&s_edges, s.edges);
    __syncthreads();
    Ctrl *c = p.ctrl;
    if (threadIdx.x == 0) {
        atomicAdd(&c->edges, s_edges);
        const uint32_t prev = __hip_atomic_fetch_add(&c->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == tm.size - 1 && p.dstats) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            Stats *st = p.dstats;
            st->status = static_cast<int32_t>(load_agent(&c->error));
            st->iterations = s.inv;
            st->items = s.items;
            st->edges = __hip_atomic_load(&c->edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st->max_frontier = s.max_in;
            st->grid = static_cast<int32_t>(tm.size);
            st->block = B;
            st->heavy_pulls = 0;
            st->frontier_edges = 0;
        }
    }
}

// Control block and counters of a fresh launch (one thread).
__global__ void pipe_init_kernel(Ctrl *c, Counters *k) {
    reset_barrier_words(c);
    c->error = 0;
    c->fatal = 0;
    c->done = 0;
    c->edges = 0;
    for (int i = 0; i < 3; ++i) {
        k->out[i] = 0;
        k->retry[i] = 0;
        k->red[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr int kSizes[] = {64, 128, 256, 512, 1024};

template <int B>
size_t lds_of(int body) {
    return body_lds<B>(body);
}

// LDS bytes of a body at workgroup size B (from its layout).
size_t body_lds_at(int body, int b) {
    switch (b) {
        case 64: return lds_of<64>(body);
        case 128: return lds_of<128>(body);
        case 256: return lds_of<256>(body);
        case 512: return lds_of<512>(body);
        default: return lds_of<1024>(body);
    }
}

bool admits(const irgl_block_constraint &k, int b, int lds_limit) {
    if (k.kind == IRGL_BLOCK_FIXED && b != k.block) return false;
    if (k.kind == IRGL_BLOCK_SHRINKABLE && b > k.block) return false;
    return static_cast<long long>(k.lds_base) + static_cast<long long>(k.lds_per_thread) * b <= lds_limit;
}

struct Layout {
    size_t ctrl, cnt, wl[3], prog, comp, hookto, minv, cmin, cfar, crev, lock, total;
};

constexpr size_t kA = 256;
constexpr size_t up(size_t x) { return (x + kA - 1) / kA * kA; }

Layout layout(int64_t n, int32_t nops, bool mst) {
    Layout L;
    const size_t nb = up(static_cast<size_t>(n) * 4);
    L.ctrl = 0;
    L.cnt = up(sizeof(Ctrl));
    L.wl[0] = L.cnt + up(sizeof(Counters));
    L.wl[1] = L.wl[0] + nb;
    L.wl[2] = L.wl[1] + nb;
    L.prog = L.wl[2] + nb;
    size_t o = L.prog + up(static_cast<size_t>(nops) * sizeof(irgl_pipe_op));
    L.comp = o;  o += mst ? nb : 0;
    L.hookto = o;  o += mst ? nb : 0;
    L.minv = o;  o += mst ? nb : 0;
    L.cmin = o;  o += mst ? up(static_cast<size_t>(n) * 8) : 0;
    L.cfar = o;  o += mst ? nb : 0;
    L.crev = o;  o += mst ? nb : 0;
    L.lock = o;  o += mst ? nb : 0;
    L.total = o;
    return L;
}

#define PIPE_HIP(call)                                                  \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return irgl_shared::note_hip_failure(e_); \
    } while (0)

template <int B>
irgl_status launch(Params &p, int dev, int requested, hipStream_t s) {
    int cus = 0, per_cu = 0;
    PIPE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    PIPE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<B>, B, 0));
    // at most 6 waves per SIMD are co-resident on gfx950 (the library's cap
    // for every cooperative launch)
    per_cu = std::min(per_cu, std::max(1, 24 / (B / kWave)));
    const int limit = per_cu * cus;
    if (limit <= 0 || requested < 0 || requested > limit) return IRGL_ERR_CONFIG;
    const int grid = requested ? requested : limit;
    void *args[] = {&p};
    PIPE_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(pipe_kernel<B>), dim3(grid), dim3(B), args, 0, s));
    return IRGL_OK;
}

int lds_limit_of_device() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return v;
}

}  // namespace pipe
}  // namespace irgl

using namespace irgl::pipe;

extern "C" {

irgl_status irgl_control_block(const irgl_block_constraint *k, int32_t nk, int32_t lds_limit, int32_t *block) {
    if ((!k && nk > 0) || nk < 0 || !block || lds_limit <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    int best = 0;
    for (int b : kSizes) {
        bool all = true;
        for (int32_t i = 0; i < nk && all; ++i) all = admits(k[i], b, lds_limit);
        if (all) best = b;  // sizes ascend: keep the highest
    }
    if (!best) return IRGL_ERR_CONFIG;
    *block = best;
    return IRGL_OK;
}

irgl_status irgl_pipe_body_constraint(int32_t body, irgl_block_constraint *out) {
    if (!out || body < 0 || body >= IRGL_BODY_COUNT) return IRGL_ERR_INVALID_ARGUMENT;
    const BodyInfo bi = body_info(body);
    // LDS grows linearly with the size (per-thread windows, per-wavefront
    // queues): the slope and intercept from the layout at 64 and 1024
    const long long l64 = static_cast<long long>(body_lds_at(body, 64));
    const long long l1024 = static_cast<long long>(body_lds_at(body, 1024));
    const long long per = (l1024 - l64 + 959) / 960;
    out->kind = bi.kind;
    out->block = bi.block;
    out->lds_per_thread = static_cast<int32_t>(per);
    out->lds_base = static_cast<int32_t>(std::max(0ll, l64 - per * 64));
    return IRGL_OK;
}

irgl_status irgl_pipe_check(const irgl_pipe_op *prog, int32_t nops) {
    if (!prog || nops <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    int stack[kDepth];
    bool invokes[kDepth];
    int sp = 0;
    for (int32_t pc = 0; pc < nops; ++pc) {
        const irgl_pipe_op &o = prog[pc];
        switch (o.op) {
            case IRGL_PIPE_INVOKE:
            case IRGL_PIPE_ITERATE: {
                if (o.a < 0 || o.a >= IRGL_BODY_COUNT) return IRGL_ERR_INVALID_ARGUMENT;
                const BodyInfo bi = body_info(o.a);
                if (o.op == IRGL_PIPE_ITERATE && !bi.uses_wl && !bi.reduces) return IRGL_ERR_INVALID_ARGUMENT;
                for (int i = 0; i < sp; ++i) invokes[i] = invokes[i] || bi.uses_wl;
                break;
            }
            case IRGL_PIPE_BEGIN:
                if (sp == kDepth || (o.a != 0 && o.a != 1)) return IRGL_ERR_INVALID_ARGUMENT;
                stack[sp] = pc;
                invokes[sp] = false;
                ++sp;
                break;
            case IRGL_PIPE_END:
                if (sp == 0) return IRGL_ERR_INVALID_ARGUMENT;
                --sp;
                // a looping Pipe must invoke a worklist body, or `in` never changes
                if (prog[stack[sp]].a == 0 && !invokes[sp]) return IRGL_ERR_INVALID_ARGUMENT;
                break;
            case IRGL_PIPE_IF: {
                const int c = o.a & ~IRGL_COND_NOT;
                if (c < IRGL_COND_IN_EMPTY || c > IRGL_COND_RETURNED) return IRGL_ERR_INVALID_ARGUMENT;
                if (o.b <= pc || o.b > nops) return IRGL_ERR_INVALID_ARGUMENT;
                break;
            }
            case IRGL_PIPE_JUMP:
                if (o.a <= pc || o.a > nops) return IRGL_ERR_INVALID_ARGUMENT;
                break;
            case IRGL_PIPE_INIT_SOURCE: break;
            default: return IRGL_ERR_INVALID_ARGUMENT;
        }
    }
    (void)stack;
    return sp == 0 ? IRGL_OK : IRGL_ERR_INVALID_ARGUMENT;
}

irgl_status irgl_pipe_control_block(const irgl_pipe_op *prog, int32_t nops, int32_t requested, int32_t lds_limit,
                                    int32_t *block) {
    irgl_status st = irgl_pipe_check(prog, nops);
    if (st) return st;
    if (!block) return IRGL_ERR_INVALID_ARGUMENT;
    if (lds_limit == 0) lds_limit = lds_limit_of_device();
    if (lds_limit <= 0) return IRGL_ERR_NO_DEVICE;
    irgl_block_constraint ks[IRGL_BODY_COUNT + 1];
    int nk = 0;
    bool seen[IRGL_BODY_COUNT] = {};
    for (int32_t pc = 0; pc < nops; ++pc) {
        const irgl_pipe_op &o = prog[pc];
        if ((o.op == IRGL_PIPE_INVOKE || o.op == IRGL_PIPE_ITERATE) && !seen[o.a]) {
            seen[o.a] = true;
            irgl_pipe_body_constraint(o.a, &ks[nk++]);
        }
    }
    if (requested) {
        // the caller's size is one more constraint: a FixedBlock of that size
        ks[nk++] = irgl_block_constraint{IRGL_BLOCK_FIXED, requested, 0, 0};
    }
    return irgl_control_block(ks, nk, lds_limit, block);
}

static bool uses(const irgl_pipe_op *prog, int32_t nops, bool mst) {
    for (int32_t pc = 0; pc < nops; ++pc)
        if ((prog[pc].op == IRGL_PIPE_INVOKE || prog[pc].op == IRGL_PIPE_ITERATE) && body_info(prog[pc].a).mst == mst)
            return true;
    return false;
}

irgl_status irgl_pipe_workspace_bytes(irgl_graph g, const irgl_pipe_op *prog, int32_t nops, size_t *bytes) {
    int dev = 0;
    irgl_csr csr;
    irgl_status st = irgl_shared::caller_csr(g, &dev, &csr);
    if (st) return st;
    st = irgl_pipe_check(prog, nops);
    if (st) return st;
    if (!bytes) return IRGL_ERR_INVALID_ARGUMENT;
    *bytes = layout(csr.n, nops, uses(prog, nops, true)).total;
    return IRGL_OK;
}

irgl_status irgl_pipe_run(irgl_graph g, const irgl_pipe_op *prog, int32_t nops, const irgl_pipe_io *io, void *ws,
                          size_t ws_bytes, void *stream, irgl_stats *dstats) {
    int dev = 0;
    irgl_csr csr;
    irgl_status st = irgl_shared::caller_csr(g, &dev, &csr);
    if (st) return st;
    st = irgl_pipe_check(prog, nops);
    if (st) return st;
    if (!io || !ws) return IRGL_ERR_INVALID_ARGUMENT;
    bool init_source = false, bfs = false, pull = false;
    for (int32_t pc = 0; pc < nops; ++pc) {
        if (prog[pc].op == IRGL_PIPE_INIT_SOURCE) init_source = true;
        if (prog[pc].op == IRGL_PIPE_INVOKE || prog[pc].op == IRGL_PIPE_ITERATE) {
            bfs |= body_info(prog[pc].a).bfs;
            pull |= prog[pc].a == IRGL_BODY_BFS_PULL;
        }
    }
    const bool mst = uses(prog, nops, true);
    if ((bfs || init_source) && (!io->level || io->src < 0 || io->src >= csr.n)) return IRGL_ERR_INVALID_ARGUMENT;
    if (mst && (!io->component || !io->weight || (csr.m > 0 && !io->in_forest))) return IRGL_ERR_INVALID_ARGUMENT;
    if ((pull || mst) && !(csr.flags & IRGL_SYMMETRIC)) return IRGL_ERR_CONFIG;
    if (mst && !csr.w && csr.m > 0) return IRGL_ERR_NO_WEIGHTS;
    if (io->trace_len && !io->trace) return IRGL_ERR_INVALID_ARGUMENT;
    int cur = -1;
    PIPE_HIP(hipGetDevice(&cur));
    if (cur != dev) PIPE_HIP(hipSetDevice(dev));
    int32_t block = 0;
    st = irgl_pipe_control_block(prog, nops, io->block, 0, &block);
    const Layout L = layout(csr.n, nops, mst);
    if (st == IRGL_OK && ws_bytes < L.total) st = IRGL_ERR_WORKSPACE_TOO_SMALL;
    int khz = 0;
    if (st == IRGL_OK && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        st = irgl_shared::note_hip_failure(hipGetLastError());
    if (st) {
        if (cur != dev) (void)hipSetDevice(cur);
        return st;
    }
    if (khz <= 0) khz = 100000;
    char *b = static_cast<char *>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Params p;
    std::memset(&p, 0, sizeof(p));
    p.n = csr.n;
    p.m = csr.m;
    p.row_ptr = csr.row_ptr;
    p.col = csr.col;
    p.w = csr.w;
    p.prog = reinterpret_cast<const irgl_pipe_op *>(b + L.prog);
    p.nops = nops;
    p.src = io->src;
    p.ctrl = reinterpret_cast<irgl::Ctrl *>(b + L.ctrl);
    p.cnt = reinterpret_cast<Counters *>(b + L.cnt);
    for (int i = 0; i < 3; ++i) p.wl[i] = reinterpret_cast<int32_t *>(b + L.wl[i]);
    p.cap = static_cast<uint32_t>(csr.n);
    p.level = io->level;
    if (mst) {
        p.comp = reinterpret_cast<int32_t *>(b + L.comp);
        p.hookto = reinterpret_cast<int32_t *>(b + L.hookto);
        p.minv = reinterpret_cast<int32_t *>(b + L.minv);
        p.cmin = reinterpret_cast<unsigned long long *>(b + L.cmin);
        p.cfar = reinterpret_cast<int32_t *>(b + L.cfar);
        p.crev = reinterpret_cast<int32_t *>(b + L.crev);
        p.lock = reinterpret_cast<uint32_t *>(b + L.lock);
        p.component = io->component;
        p.in_forest = io->in_forest;
        p.weight = reinterpret_cast<unsigned long long *>(io->weight);
    }
    p.trace = io->trace;
    p.trace_len = io->trace ? io->trace_len : 0u;
    p.max_inv = io->max_invocations ? io->max_invocations
                                    : static_cast<uint32_t>(std::min<int64_t>(0x7FFFFFF0ll, 8ll * csr.n + 64));
    const uint32_t wd_ms = io->watchdog_ms ? io->watchdog_ms : 20000u;
    p.wd_ticks = static_cast<unsigned long long>(wd_ms) * static_cast<unsigned long long>(khz);
    p.barrier = IRGL_BARRIER_XCD;
    p.force_retry = io->force_retry;
    p.dstats = reinterpret_cast<irgl::Stats *>(dstats);
    hipError_t e = hipMemcpyAsync(b + L.prog, prog, static_cast<size_t>(nops) * sizeof(irgl_pipe_op),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pipe_init_kernel, dim3(1), dim3(1), 0, s, p.ctrl, p.cnt);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        st = irgl_shared::note_hip_failure(e);
    } else {
        switch (block) {
            case 64: st = launch<64>(p, dev, io->grid, s); break;
            case 128: st = launch<128>(p, dev, io->grid, s); break;
            case 256: st = launch<256>(p, dev, io->grid, s); break;
            case 512: st = launch<512>(p, dev, io->grid, s); break;
            default: st = launch<1024>(p, dev, io->grid, s); break;
        }
    }
    if (cur != dev) (void)hipSetDevice(cur);
    return st;
}

}  // extern "C"
