// Boruvka minimum spanning forest: the workload the paper uses to show the
// Atomic construct (Section 3, the find-minimum-cross-component-edge kernel).
//
// Every vertex starts as its own component.  A round is three phases of one
// persistent cooperative launch, separated by the grid barrier:
//   1. find-min-edge: a ForAll over the worklist (all vertices in round 0,
//      then the vertices that still had a cross-component edge, the kernel's
//      Retry-style re-push) finds each vertex's lightest edge to another
//      component and makes it its component's candidate inside an atomic
//      section;
//   2. every component root hooks to the component at the other end of its
//      chosen edge and emits that edge into the forest (a pair of components
//      that chose the same edge keeps the smaller id as root and emits the
//      edge once);
//   3. pointer jumping flattens the hooks (iterated while Any(changed), with
//      the block-aggregated reduction), and every vertex moves to its new root.
// The loop ends when a round's worklist is empty.
//
// Edges are compared in the total order (weight, smaller endpoint, larger
// endpoint), so the minimum forest is unique and no cycle can form.  An
// undirected edge {u, v} is named by its canonical entry: the CSR index of
// the u -> v entry with u < v; (weight << 32 | canonical entry) is then a
// 64-bit key in the same order (entries of a row are sorted by destination).
//
// The atomic section updates two words of the component, its lightest
// weight and its edge, together.  Three compilations of it (IRGL_LOCK_*):
//   packed  - the MI355X form: the two words are one 64-bit key, updated
//             with a single 64-bit atomicMin;
//   spin    - the blocking Atomic: a compare-and-swap lock per component in
//             a divergence-safe retry loop (the lock holder runs its section
//             and releases inside the same loop iteration, so lanes of one
//             wavefront waiting on each other cannot deadlock);
//   ticket  - the same section under a ticket lock.
// Before taking a lock a lane reads the component's weight: weights only
// fall during phase 1, so a candidate heavier than a stale read cannot win.
// The lanes of a wavefront that offer to the same component first reduce
// their candidates to one (cooperative conversion, Sections 3.5 and 4.2,
// applied to the atomic section), so a giant component sees one lock
// acquisition or atomic per wavefront instead of one per vertex.
// Every lock wait is bounded by a wall-clock limit (IRGL_ERR_WATCHDOG).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "irgl.h"
#include "irgl_device.h"

namespace irgl_shared {
irgl_status note_hip_failure(hipError_t e);
irgl_status caller_csr(const irgl_graph_s *g, int *device, irgl_csr *out);
}  // namespace irgl_shared

namespace irgl {
namespace mst {

constexpr unsigned long long kNoKey = ~0ull;
constexpr int kTBlock = 4096;   // ... this many or more: the whole workgroup
constexpr int kMstQueue = 256;  // LDS push staging per wavefront

struct MstParams {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    int32_t *comp;               // component (root id) of every vertex
    int32_t *hook;               // per root: the root it joins this round
    unsigned long long *key;     // packed: per root, weight << 32 | canonical entry
    uint32_t *minwt;             // spin / ticket: per root, the weight ...
    int32_t *minedge;            // ... and the canonical entry of its chosen edge
    uint32_t *lock;              // spin: per root lock word
    uint32_t *ticket;            // ticket: per root next ticket ...
    uint32_t *serving;           // ... and the ticket being served
    int32_t *wl0, *wl1;          // worklists of vertices that still had a cross edge
    int32_t *forest;             // emitted forest edges (canonical entries), capacity n
    int32_t *repmin;             // per root: smallest vertex id of its tree
    uint8_t *in_forest;          // optional: per CSR entry, 1 for both directions of forest edges
    int32_t *comp_out;           // optional: smallest vertex id of each vertex's tree
    unsigned long long *weight;  // forest weight (device)
    Ctrl *ctrl;
    Stats *dstats;
    uint32_t lock_kind;
    uint32_t max_rounds;
    unsigned long long wd_ticks;
    unsigned long long spin_ticks;
    uint32_t barrier;
};

// The launch reuses control-block counters: cnt[] for the rotating worklist
// counts, red[] for the pointer-jumping reduction, bu_scan for the number of
// emitted forest edges.
__device__ __forceinline__ unsigned long long *forest_count(Ctrl *c) { return &c->bu_scan; }

template <int B>
struct MstSmem {
    static constexpr int NW = B / kWave;
    int queue[NW][kMstQueue];
    int fill[NW];
    uint32_t base;
    int flag;
    int owner;
    int big_v, big_r0, big_r1;
    unsigned long long red[NW];
    unsigned long long wsum[NW];
    int dsum[NW];
    // gather tier: the workgroup's rows concatenated (exclusive scan of the
    // degrees), each slot's owner found by a binary search
    int gstart[B];
    int gr0[B];
    int gv[B];
    int gc[B];
    unsigned long long vmin[B];  // per row: lightest cross edge as (w << 32 | neighbour)
};

// For a fixed vertex v, ordering its edges {v, u} by (w, smaller endpoint,
// larger endpoint) is ordering them by (w, u): an edge to u < v has the
// smaller endpoint u < v, an edge to u > v has v.  So a row's lightest cross
// edge is the minimum of the 64-bit row key w << 32 | u.

// Row key minimum of entries [r0, r1) of vertex v in component c, entries
// first, first + step, ...
__device__ __forceinline__ unsigned long long scan_row(const MstParams &p, int v, int c, int r0, int r1, int first,
                                                       int step, unsigned long long &scanned) {
    unsigned long long b = kNoKey;
    for (int e = r0 + first; e < r1; e += step) {
        const int u = p.col[e];
        ++scanned;
        if (u == v || p.comp[u] == c) continue;
        b = min(b, (static_cast<unsigned long long>(p.w[e]) << 32) | static_cast<uint32_t>(u));
    }
    return b;
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long b) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) b = min(b, static_cast<unsigned long long>(__shfl_xor(b, off, kWave)));
    return b;
}

// The entry u -> v of u's row (rows sorted by destination: binary search,
// then a linear scan if the row is not sorted), or -1.
__device__ __forceinline__ int find_entry(const MstParams &p, int u, int v) {
    int a = p.row_ptr[u], b = p.row_ptr[u + 1];
    const int r0 = a, r1 = b;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (p.col[mid] < v) a = mid + 1;
        else b = mid;
    }
    if (a < r1 && p.col[a] == v) return a;
    for (int e = r0; e < r1; ++e)
        if (p.col[e] == v) return e;
    return -1;
}

// The row (source vertex) of CSR entry e.
__device__ __forceinline__ int row_of(const MstParams &p, int e) {
    int a = 0, b = p.n;  // largest v with row_ptr[v] <= e
    while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (p.row_ptr[mid] <= e) a = mid;
        else b = mid;
    }
    return a;
}

// Candidate key (weight << 32 | canonical entry) of row key rk of vertex v,
// or kNoKey.  The canonical entry is the smaller endpoint's entry.
__device__ __forceinline__ unsigned long long candidate_key(const MstParams &p, int v, unsigned long long rk) {
    if (rk == kNoKey) return kNoKey;
    const int u = static_cast<int>(rk & 0xFFFFFFFFull);
    const int canon = find_entry(p, min(u, v), max(u, v));
    if (canon < 0) {  // no reverse entry: the CSR is not symmetric
        set_error(p.ctrl, IRGL_ERR_INVALID_GRAPH, false);
        return kNoKey;
    }
    return (rk & 0xFFFFFFFF00000000ull) | static_cast<uint32_t>(canon);
}

// The atomic section of find-min-edge: make `k` the candidate of component
// c if it is lighter.  Called by every lane; `want` says whether this lane
// has a candidate.
__device__ __forceinline__ void offer(const MstParams &p, int c, unsigned long long k, bool want) {
    if (p.lock_kind == IRGL_LOCK_PACKED) {
        if (want && k < p.key[c]) atomicMin(&p.key[c], k);
        return;
    }
    const uint32_t wt = static_cast<uint32_t>(k >> 32);
    const int32_t edge = static_cast<int32_t>(k & 0xFFFFFFFFull);
    // a candidate heavier than a (possibly stale, never lower) read cannot win
    bool pending = want && wt <= p.minwt[c];
    const bool ticket = p.lock_kind == IRGL_LOCK_TICKET;
    uint32_t mine = 0;
    if (pending && ticket) mine = atomicAdd(&p.ticket[c], 1u);
    const unsigned long long t0 = wall_clock64();
    // The loop leaves only when no lane of the wavefront is pending (a
    // wave-uniform test at the top).  With a per-lane exit the compiler may
    // legally move the section and its release after the loop, where a lane
    // holding the lock waits, masked off, for lanes of its own wavefront
    // that spin on that lock: the divergence deadlock the Atomic construct
    // exists to avoid.  Here the section runs in the iteration that took the
    // lock, before the next test.
    for (;;) {
        if (__ballot(pending) == 0ull) break;
        if (pending) {
            const bool held = ticket ? load_agent(&p.serving[c]) == mine : atomicCAS(&p.lock[c], 0u, 1u) == 0u;
            if (held) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const uint32_t cw = load_agent(&p.minwt[c]);
                const int32_t ce = static_cast<int32_t>(load_agent(reinterpret_cast<uint32_t *>(&p.minedge[c])));
                if (wt < cw || (wt == cw && (ce < 0 || edge < ce))) {
                    store_agent(&p.minwt[c], wt);
                    store_agent(reinterpret_cast<uint32_t *>(&p.minedge[c]), static_cast<uint32_t>(edge));
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (ticket) store_agent(&p.serving[c], mine + 1u);
                else store_agent(&p.lock[c], 0u);
                pending = false;
            } else if (wall_clock64() - t0 > p.spin_ticks) {
                set_error(p.ctrl, kErrWatchdog, true);
                pending = false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// The component's chosen key after phase 1 (kNoKey: none).
__device__ __forceinline__ unsigned long long chosen(const MstParams &p, int c) {
    if (p.lock_kind == IRGL_LOCK_PACKED) return p.key[c];
    const int32_t e = p.minedge[c];
    return e < 0 ? kNoKey : (static_cast<unsigned long long>(p.minwt[c]) << 32) | static_cast<uint32_t>(e);
}

template <int B>
__device__ __forceinline__ unsigned long long block_sum(MstSmem<B> &sm, unsigned long long x) {
    constexpr int NW = B / kWave;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    __syncthreads();
    if (lane_id() == 0) sm.wsum[threadIdx.x / kWave] = x;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += sm.wsum[k];
    return t;
}

// Phase 1 over worklist `in` (identity when null) of cnt_in vertices; pushes
// the vertices that have a cross edge.  Rows of kTBlock or more entries are
// scanned by the whole workgroup one at a time; the other rows of a tile are
// concatenated and dealt to the lanes in full rounds (load-balanced gather),
// each slot folding its edge into its row's minimum with an LDS atomicMin.
template <int B>
__device__ __forceinline__ void find_min_edges(const MstParams &p, MstSmem<B> &sm, Team tm, const int32_t *in,
                                               uint32_t cnt_in, WaveQueue<kMstQueue> &wq, uint32_t *cnt_out,
                                               int32_t *out, unsigned long long &scanned) {
    constexpr int NW = B / kWave;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
    for (uint32_t base = tm.id * B; base < cnt_in; base += tm.size * B) {
        const uint32_t i = base + tid;
        int v = -1, c = -1, r0 = 0, r1 = 0;
        if (i < cnt_in) {
            v = in ? in[i] : static_cast<int>(i);
            c = p.comp[v];
            r0 = p.row_ptr[v];
            r1 = p.row_ptr[v + 1];
        }
        int deg = r1 - r0;
        unsigned long long rk = kNoKey;
        // workgroup tier: one large row at a time
        while (__syncthreads_or(deg >= kTBlock)) {
            if (deg >= kTBlock) sm.owner = tid;
            __syncthreads();
            if (sm.owner == tid) {
                sm.big_v = v;
                sm.big_r0 = r0;
                sm.big_r1 = r1;
                deg = 0;
            }
            __syncthreads();
            const int bv = sm.big_v;
            const unsigned long long b = wave_min(scan_row(p, bv, p.comp[bv], sm.big_r0, sm.big_r1, tid, B, scanned));
            if (lane == 0) sm.red[wid] = b;
            __syncthreads();
            if (sm.owner == tid) {
                for (int k = 0; k < NW; ++k) rk = min(rk, sm.red[k]);
            }
            __syncthreads();
        }
        // gather tier
        const int incl = wave_inclusive_scan(deg);
        if (lane == kWave - 1) sm.dsum[wid] = incl;
        sm.vmin[tid] = kNoKey;
        __syncthreads();
        int total = 0, wpre = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            wpre += (k < wid) ? sm.dsum[k] : 0;
            total += sm.dsum[k];
        }
        sm.gstart[tid] = wpre + incl - deg;
        sm.gr0[tid] = r0;
        sm.gv[tid] = v;
        sm.gc[tid] = c;
        __syncthreads();
        for (int done = 0; done < total; done += B) {
            const int slot = done + tid;
            if (slot < total) {
                int o = 0;
#pragma unroll
                for (int step = B / 2; step > 0; step >>= 1)
                    if (sm.gstart[o + step] <= slot) o += step;
                const int e = sm.gr0[o] + (slot - sm.gstart[o]);
                const int u = p.col[e];
                ++scanned;
                if (u != sm.gv[o] && p.comp[u] != sm.gc[o])
                    atomicMin(&sm.vmin[o], (static_cast<unsigned long long>(p.w[e]) << 32) | static_cast<uint32_t>(u));
            }
        }
        __syncthreads();
        if (deg > 0) rk = sm.vmin[tid];
        unsigned long long k = v >= 0 ? candidate_key(p, v, rk) : kNoKey;
        const bool has = k != kNoKey;
        // Cooperative conversion of the atomic section: the candidates of the
        // wavefront's lanes that share the first candidate lane's component
        // (in later rounds most lanes are in one giant component) are reduced
        // to their minimum, and only that lane enters the section for them.
        bool want = has;
        const unsigned long long cm = __ballot(has);
        if (cm) {
            const int leader = __ffsll(static_cast<long long>(cm)) - 1;
            const int cl = __shfl(c, leader, kWave);
            const bool same = has && c == cl;
            const unsigned long long kk = wave_min(same ? k : kNoKey);
            if (same) {
                want = lane == leader;
                k = kk;
            }
        }
        offer(p, c, k, want);
        wq.push(has, v, cnt_out, out, static_cast<uint32_t>(p.n), p.ctrl);
        __syncthreads();  // the gather arrays are rewritten by the next tile
    }
}

template <int B>
__global__ __launch_bounds__(B) void mst_kernel(MstParams p) {
    __shared__ MstSmem<B> sm;
    const Team tm = whole_grid();
    BarrierState bs = make_barrier_state(p.wd_ticks, p.barrier);
    Ctrl *ctrl = p.ctrl;
    const int wid = threadIdx.x / kWave;
    const uint32_t n = static_cast<uint32_t>(p.n);
    const uint32_t stride = tm.size * B;
    const uint32_t gid = tm.id * B + threadIdx.x;
    const bool lead = tm.id == 0 && threadIdx.x == 0;
    unsigned long long scanned = 0, items = 0, added = 0;
    uint32_t round = 0;
    uint32_t jumps = 0;  // pointer-jumping passes so far (rotates the reduction words)
    bool ok = true;
    for (;; ++round) {
        const uint32_t cnt_in = round == 0 ? n : min(load_agent(&ctrl->cnt[round % 3]), n);
        if (cnt_in == 0) break;
        if (round >= p.max_rounds) {
            if (lead) set_error(ctrl, kErrIterLimit, false);
            break;
        }
        items += cnt_in;
        if (lead) store_agent(&ctrl->cnt[(round + 2) % 3], 0u);
        const int32_t *in = round == 0 ? nullptr : ((round & 1u) ? p.wl1 : p.wl0);
        int32_t *out = (round & 1u) ? p.wl0 : p.wl1;
        WaveQueue<kMstQueue> wq{sm.queue[wid], 0};
        // phase 1: find-min-edge with the atomic section
        find_min_edges<B>(p, sm, tm, in, cnt_in, wq, &ctrl->cnt[(round + 1) % 3], out, scanned);
        block_drain<B, kMstQueue>(wq, sm.fill, &sm.base, &ctrl->cnt[(round + 1) % 3], out, n, ctrl);
        if (!(ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm))) break;
        // phase 2: hook every root with a candidate, emit its edge (the
        // wavefront reserves its forest slots with one atomic)
        for (uint32_t base2 = tm.id * B; base2 < n; base2 += stride) {
            const uint32_t c = base2 + threadIdx.x;
            bool emit = false;
            int e = 0;
            if (c < n && p.comp[c] == static_cast<int32_t>(c)) {
                const unsigned long long k = chosen(p, static_cast<int>(c));
                if (k != kNoKey) {
                    e = static_cast<int>(k & 0xFFFFFFFFull);
                    const int lo = row_of(p, e), hi = p.col[e];
                    const int other = p.comp[lo] == static_cast<int32_t>(c) ? hi : lo;
                    const int c2 = p.comp[other];
                    const bool mutual = chosen(p, c2) == k;
                    p.hook[c] = (mutual && static_cast<int>(c) < c2) ? static_cast<int32_t>(c) : c2;
                    emit = !(mutual && static_cast<int>(c) > c2);
                    if (emit) added += static_cast<unsigned long long>(k >> 32);
                }
            }
            const unsigned long long em = __ballot(emit);
            if (em) {
                unsigned long long slot0 = 0;
                if (lane_id() == 0) slot0 = atomicAdd(forest_count(ctrl), static_cast<unsigned long long>(__popcll(em)));
                slot0 = __shfl(slot0, 0, kWave);
                const unsigned long long slot = slot0 + lane_rank(em);
                if (emit && slot < n) p.forest[slot] = e;
            }
        }
        if (!(ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm))) break;
        // phase 3: pointer jumping over the hooks, While Any(changed)
        for (uint32_t pass = 0;; ++jumps, ++pass) {
            // the hooks form a forest (edge keys strictly fall along a hook
            // chain), so its depth is below n and log2 n passes flatten it
            if (pass > p.max_rounds) {
                if (lead) set_error(ctrl, kErrInternal, false);
                ok = false;
                break;
            }
            // red[(jumps + 1) % 3] was last read after pass jumps - 2, before
            // the barrier of pass jumps - 1; it is next set in pass jumps + 1
            uint32_t *red = &ctrl->red[jumps % 3];
            if (lead) store_agent(&ctrl->red[(jumps + 1) % 3], 0u);
            bool changed = false;
            for (uint32_t c = gid; c < n; c += stride) {
                if (p.comp[c] != static_cast<int32_t>(c)) continue;
                const int32_t h = p.hook[c];
                const int32_t hh = p.hook[h];
                if (hh != h) {
                    p.hook[c] = hh;
                    changed = true;
                }
            }
            if (__syncthreads_or(changed) && threadIdx.x == 0) atomicOr(red, 1u);
            if (!(ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm))) break;
            if (load_agent(red) == 0u) {
                ++jumps;
                break;
            }
        }
        if (!ok) break;
        // every vertex joins its new root; the roots' candidates are cleared
        for (uint32_t v = gid; v < n; v += stride) {
            p.comp[v] = p.hook[p.comp[v]];
            if (p.lock_kind == IRGL_LOCK_PACKED) {
                p.key[v] = kNoKey;
            } else {
                p.minwt[v] = kInf;
                p.minedge[v] = -1;
            }
        }
        if (!(ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm))) break;
        // (a root's hook is itself again: roots that kept their id were the
        // hook forest's roots)
    }
    const unsigned long long wsum = block_sum<B>(sm, added);
    const unsigned long long ssum = block_sum<B>(sm, scanned);
    if (threadIdx.x == 0) {
        if (wsum) atomicAdd(p.weight, wsum);
        atomicAdd(&ctrl->edges, ssum);
        if (tm.id == 0) {
            ctrl->iterations = round;
            ctrl->items = items;
        }
    }
    if (ok) ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm);
    if (ok) {
        // smallest vertex id of every tree, then the per-entry marks
        // (consecutive lanes hold consecutive ids: the first lane of each run
        // of one component holds its smallest id in the wavefront)
        for (uint32_t base3 = tm.id * B; base3 < n; base3 += stride) {
            const uint32_t v = base3 + threadIdx.x;
            const bool live = v < n;
            const int cv = live ? p.comp[v] : -1;
            const unsigned long long lm = __ballot(live);
            bool mine = live;
            if (lm) {
                const int leader = __ffsll(static_cast<long long>(lm)) - 1;
                const int cl = __shfl(cv, leader, kWave);
                if (live && cv == cl && lane_id() != leader) mine = false;
            }
            if (mine) atomicMin(&p.repmin[cv], static_cast<int32_t>(v));
        }
        const unsigned long long nf = min(__hip_atomic_load(forest_count(ctrl), __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT),
                                          static_cast<unsigned long long>(n));
        if (p.in_forest) {
            for (unsigned long long k = gid; k < nf; k += stride) {
                const int e = p.forest[k];
                const int lo = row_of(p, e), hi = p.col[e];
                p.in_forest[e] = 1;
                const int r = find_entry(p, hi, lo);
                if (r >= 0) p.in_forest[r] = 1;
            }
        }
        ok = grid_barrier(ctrl, bs, &sm.flag, nullptr, tm);
        if (ok && p.comp_out)
            for (uint32_t v = gid; v < n; v += stride) p.comp_out[v] = p.repmin[p.comp[v]];
    }
    // statistics: the last workgroup to leave publishes them
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(&ctrl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == tm.size - 1 && p.dstats) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            Stats *s = p.dstats;
            s->status = static_cast<int32_t>(load_agent(&ctrl->error));
            s->iterations = ctrl->iterations;
            s->items = ctrl->items;
            s->edges = __hip_atomic_load(&ctrl->edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s->max_frontier = 0;
            s->grid = static_cast<int32_t>(tm.size);
            s->block = B;
            s->heavy_pulls = 0;
            s->frontier_edges = __hip_atomic_load(forest_count(ctrl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void mst_init_kernel(MstParams p, unsigned long long m) {
    const unsigned long long stride = static_cast<unsigned long long>(gridDim.x) * blockDim.x;
    const unsigned long long t = static_cast<unsigned long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (unsigned long long v = t; v < static_cast<unsigned long long>(p.n); v += stride) {
        p.comp[v] = static_cast<int32_t>(v);
        p.hook[v] = static_cast<int32_t>(v);
        p.key[v] = kNoKey;
        p.minwt[v] = kInf;
        p.minedge[v] = -1;
        p.lock[v] = 0;
        p.ticket[v] = 0;
        p.serving[v] = 0;
        p.repmin[v] = 0x7FFFFFFF;
    }
    if (p.in_forest)
        for (unsigned long long e = t; e < m; e += stride) p.in_forest[e] = 0;
    if (t == 0) {
        Ctrl *c = p.ctrl;
        for (int k = 0; k < 3; ++k) {
            c->cnt[k] = 0;
            c->red[k] = 0;
        }
        c->bu_scan = 0;
        reset_barrier_words(c);
        c->error = 0;
        c->fatal = 0;
        c->done = 0;
        c->iterations = 0;
        c->items = 0;
        c->edges = 0;
        *p.weight = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlignB = 256;
constexpr size_t align_b(size_t x) { return (x + kAlignB - 1) / kAlignB * kAlignB; }

struct MstLayout {
    size_t ctrl, comp, hook, key, minwt, minedge, lock, ticket, serving, wl0, wl1, forest, repmin, weight, total;
};

MstLayout mst_layout(int64_t n) {
    MstLayout L;
    const size_t nb = align_b(static_cast<size_t>(n) * 4);
    L.ctrl = 0;
    L.comp = align_b(sizeof(Ctrl));
    L.hook = L.comp + nb;
    L.key = L.hook + nb;
    L.minwt = L.key + align_b(static_cast<size_t>(n) * 8);
    L.minedge = L.minwt + nb;
    L.lock = L.minedge + nb;
    L.ticket = L.lock + nb;
    L.serving = L.ticket + nb;
    L.wl0 = L.serving + nb;
    L.wl1 = L.wl0 + nb;
    L.forest = L.wl1 + nb;
    L.repmin = L.forest + nb;
    L.weight = L.repmin + nb;
    L.total = L.weight + kAlignB;
    return L;
}

#define MST_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return irgl_shared::note_hip_failure(e_); \
    } while (0)

template <int B>
irgl_status mst_grid(int dev, int requested, int *grid) {
    int cus = 0, per_cu = 0;
    MST_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MST_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mst_kernel<B>, B, 0));
    // at most 6 waves per SIMD are co-resident on gfx950 (the same cap as
    // every other cooperative launch of the library)
    per_cu = std::min(per_cu, std::max(1, 24 / (B / kWave)));
    const int limit = per_cu * cus;
    if (limit <= 0 || requested < 0 || requested > limit) return IRGL_ERR_CONFIG;
    *grid = requested ? requested : limit;
    return IRGL_OK;
}

template <int B>
irgl_status mst_launch(MstParams &p, int dev, int requested, hipStream_t s) {
    int grid = 0;
    irgl_status st = mst_grid<B>(dev, requested, &grid);
    if (st) return st;
    void *args[] = {&p};
    MST_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(mst_kernel<B>), dim3(grid), dim3(B), args, 0,
                                       s));
    return IRGL_OK;
}

}  // namespace mst
}  // namespace irgl

using namespace irgl::mst;

extern "C" {

irgl_status irgl_mst_workspace_bytes(irgl_graph g, size_t *bytes) {
    int dev = 0;
    irgl_csr csr;
    irgl_status st = irgl_shared::caller_csr(g, &dev, &csr);
    if (st) return st;
    if (!bytes) return IRGL_ERR_INVALID_ARGUMENT;
    *bytes = mst_layout(csr.n).total;
    return IRGL_OK;
}

irgl_status irgl_mst(irgl_graph g, uint64_t *weight, int32_t *component, uint8_t *in_forest, void *ws,
                     size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_mst_config *cfg) {
    int dev = 0;
    irgl_csr csr;
    irgl_status st = irgl_shared::caller_csr(g, &dev, &csr);
    if (st) return st;
    if (!weight || !ws) return IRGL_ERR_INVALID_ARGUMENT;
    if (!csr.w && csr.m > 0) return IRGL_ERR_NO_WEIGHTS;  // an edgeless graph needs none
    // 512 measured fastest on RMAT-22 (25.4 ms against 26.9 at 256 and 25.6 at 1024)
    const int block = (cfg && cfg->block) ? cfg->block : 512;
    if (block != 256 && block != 512 && block != 1024) return IRGL_ERR_CONFIG;
    const uint32_t kind = cfg ? cfg->lock : IRGL_LOCK_PACKED;
    if (kind > IRGL_LOCK_TICKET) return IRGL_ERR_CONFIG;
    const uint32_t barrier = cfg ? cfg->barrier : IRGL_BARRIER_XCD;
    if (barrier > IRGL_BARRIER_WORKGROUP) return IRGL_ERR_CONFIG;
    if (csr.m >= (1ll << 31)) return IRGL_ERR_TOO_LARGE;  // canonical entries are 31-bit
    const MstLayout L = mst_layout(csr.n);
    if (ws_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    int cur = -1;
    MST_HIP(hipGetDevice(&cur));
    if (cur != dev) MST_HIP(hipSetDevice(dev));
    int khz = 0;
    MST_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) khz = 100000;
    char *base = static_cast<char *>(ws);
    MstParams p;
    std::memset(&p, 0, sizeof(p));
    p.n = csr.n;
    p.row_ptr = csr.row_ptr;
    p.col = csr.col;
    p.w = csr.w;
    p.comp = reinterpret_cast<int32_t *>(base + L.comp);
    p.hook = reinterpret_cast<int32_t *>(base + L.hook);
    p.key = reinterpret_cast<unsigned long long *>(base + L.key);
    p.minwt = reinterpret_cast<uint32_t *>(base + L.minwt);
    p.minedge = reinterpret_cast<int32_t *>(base + L.minedge);
    p.lock = reinterpret_cast<uint32_t *>(base + L.lock);
    p.ticket = reinterpret_cast<uint32_t *>(base + L.ticket);
    p.serving = reinterpret_cast<uint32_t *>(base + L.serving);
    p.wl0 = reinterpret_cast<int32_t *>(base + L.wl0);
    p.wl1 = reinterpret_cast<int32_t *>(base + L.wl1);
    p.forest = reinterpret_cast<int32_t *>(base + L.forest);
    p.repmin = reinterpret_cast<int32_t *>(base + L.repmin);
    p.in_forest = in_forest;
    p.comp_out = component;
    p.weight = reinterpret_cast<unsigned long long *>(weight);
    p.ctrl = reinterpret_cast<irgl::Ctrl *>(base + L.ctrl);
    p.dstats = reinterpret_cast<irgl::Stats *>(dstats);
    p.lock_kind = kind;
    // components at least halve every round: ceil(log2 n) + 2 rounds suffice
    uint32_t rounds = 2;
    for (int64_t x = 1; x < csr.n; x <<= 1) ++rounds;
    p.max_rounds = rounds;
    const uint32_t wd_ms = (cfg && cfg->watchdog_ms) ? cfg->watchdog_ms : 20000u;
    p.wd_ticks = static_cast<unsigned long long>(wd_ms) * static_cast<unsigned long long>(khz);
    p.spin_ticks = p.wd_ticks;
    p.barrier = barrier;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned long long m = static_cast<unsigned long long>(csr.m);
    const int fill = static_cast<int>(std::min<int64_t>(65535, (std::max<int64_t>(csr.n, csr.m) + 255) / 256));
    hipLaunchKernelGGL(mst_init_kernel, dim3(std::max(fill, 1)), dim3(256), 0, s, p, m);
    MST_HIP(hipGetLastError());
    switch (block) {
        case 256: st = mst_launch<256>(p, dev, cfg ? cfg->grid : 0, s); break;
        case 512: st = mst_launch<512>(p, dev, cfg ? cfg->grid : 0, s); break;
        default: st = mst_launch<1024>(p, dev, cfg ? cfg->grid : 0, s); break;
    }
    if (cur != dev) (void)hipSetDevice(cur);
    return st;
}

}  // extern "C"
