// Host runtime and C ABI of the MI355X BFS/SSSP library (declared in
// include/irgl.h).  It owns no device memory: graphs are borrowed caller
// arrays, per-query state lives in a caller workspace.  It picks block sizes
// and tier thresholds, sizes the co-resident grid with the occupancy API
// (Section 3.4: a grid barrier is safe only when every workgroup is
// resident), and launches either the outlined persistent loop (one
// cooperative launch per query) or the un-outlined host loop.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "irgl.h"
#include "irgl_kernels.h"
#include "irgl_batch.h"

using namespace irgl;

static_assert(sizeof(Stats) == sizeof(irgl_stats), "irgl_stats layout");
static_assert(offsetof(Stats, edges) == offsetof(irgl_stats, edges), "irgl_stats layout");
static_assert(offsetof(Stats, block) == offsetof(irgl_stats, block), "irgl_stats layout");

struct irgl_batch_s {
    int32_t ntasks;
    hipStream_t stream;
    hipEvent_t done;
    void *host_tasks;   // pinned staging of the task table
    Stats *dev_stats;   // per-task statistics in the workspace
    bool waited;
};

struct irgl_server_s {
    int device;
    hipStream_t stream;
    hipEvent_t ran;          // recorded after each server launch
    bool launched;
    int block, grid;
    irgl_batch_config cfg;
    uint32_t delta;
    int32_t ring_cap;
    uint64_t next_ticket;
    unsigned long long *dev_head;  // device: claimed | gangs << 32 | pending << 63
    Stats *dev_stats;        // device: per ring slot statistics
    bool sssp_ok;            // scratch includes the SSSP arrays
    int64_t small_n, small_m;  // team regions are sized for these (graphs below gang_edges)
    int64_t gang_n, gang_m;    // the gang region is sized for these
    uint32_t gang_edges;
    uint32_t gang_queue;
    uint64_t completed;        // tickets polled done
    void *host_mem;          // pinned: ring | tail | stop | done[] | stats[]
    void *params;            // ServerParams (host copy reused for launches)
    uint64_t *acked;         // per ring slot: 1 + the last ticket polled as done
    uint64_t launches;       // server kernel launches so far
};

struct irgl_graph_s {
    int32_t n;
    int64_t m;
    const int32_t *row_ptr;   // the arrays single queries traverse (relabelled copy, if any)
    const int32_t *col;
    const uint32_t *w;
    uint32_t flags;
    int device;
    uint64_t weight_sum;  // from IRGL_VALIDATE, else 0
    uint32_t max_degree;  // largest out-degree, from IRGL_VALIDATE, else 0
    // caller's arrays (batched and served tasks traverse these)
    const int32_t *orig_row_ptr;
    const int32_t *orig_col;
    const uint32_t *orig_w;
    // degree-sorted relabelling (irgl_graph_upload_reordered), else null / empty
    const int32_t *perm;           // device: internal id -> caller id
    const int32_t *inv;            // device: caller id -> internal id
    std::vector<int32_t> inv_host;  // host: caller id -> internal id
    // SSSP copy of a relabelled weighted graph (null otherwise): the rows of
    // (col, w) partitioned into the edges lighter than split_delta, then the
    // rest, each part in id order; split[v] = first heavy edge of row v.
    // `split` is null when no edge is heavy (the partition would be unused).
    int32_t *scol = nullptr;
    uint32_t *sw = nullptr;
    int32_t *split_store = nullptr;
    const int32_t *split = nullptr;
    uint32_t split_delta = IRGL_DELTA_NONE;
    unsigned long long heavy_m = 0;  // heavy entries of the partition
    // SSSP near/far step of single queries that leave it at 0
    uint32_t qdelta = IRGL_DELTA_NONE;
};

namespace {

thread_local int32_t g_last_hip_error = 0;

irgl_status hip_fail(hipError_t e) {
    g_last_hip_error = static_cast<int32_t>(e);
    (void)hipGetLastError();  // clear the sticky per-thread error
    return IRGL_ERR_DEVICE;
}

#define IRGL_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_);       \
    } while (0)

static_assert(kBarXcd == IRGL_BARRIER_XCD && kBarWorkgroup == IRGL_BARRIER_WORKGROUP, "barrier scheme values");
constexpr size_t kAlign = 256;

// Default bitmap refresh point: a refresh scans all n vertices, so it pays
// once the vertices reached since the previous refresh carry about n/2
// edges, i.e. after n^2 / (2m) new vertices (at mean degree m/n).
uint32_t default_t_bitmap(int64_t n, int64_t m) {
    if (m <= 0) return static_cast<uint32_t>(std::max<int64_t>(1, n));
    const double t = static_cast<double>(n) * static_cast<double>(n) / (2.0 * static_cast<double>(m));
    return static_cast<uint32_t>(std::max(1.0, std::min(static_cast<double>(n), t)));
}
// Default SSSP near/far step, from the graph's shape (weights >= 1):
// * mean degree below kDeltaMinDegree (road-like, high diameter): plain
//   Bellman-Ford rescans long chains many times; the step is kDeltaScale x
//   mean weight / mean degree;
// * denser and near-regular (largest out-degree at most kSkew x the mean):
//   plain order still re-relaxes every edge 4-6 times; the step is
//   kDeltaDenseScale x mean weight / mean degree;
// * denser and scale-free (hubs): plain order re-relaxes ~3 times per edge,
//   and each near/far step adds a grid barrier per extra invocation; the
//   saved relaxations repay the barriers only on large graphs (at least
//   kDeltaSkewMinEdges edges), where the step is the mean weight.
constexpr double kDeltaScale = 32.0;
constexpr double kDeltaDenseScale = 16.0;
constexpr double kDeltaMinDegree = 8.0;
constexpr double kSkew = 16.0;
constexpr int64_t kDeltaSkewMinEdges = int64_t(1) << 26;

uint32_t default_delta(const irgl_graph_s *g);
uint32_t delta_rule(const irgl_graph_s *g, bool partitioned);
// The scale-free branch of the rule (mean degree at least kDeltaMinDegree,
// largest out-degree above kSkew times the mean), from the validation pass.
bool scale_free(const irgl_graph_s *g);
// Far-list divisor of the bucketing's early end on split scale-free graphs:
// it ends once the far list holds fewer than (items popped so far) /
// kTailDiv vertices.  Re-derived once an expansion without a threshold
// relaxes whole rows (no heavy pass left), with the step W/8 and the
// threshold growth (32 sources, ms per query at divisors 16 / 4 / 2 / 1,
// and at 1 with the far list compared against 2 / 4 / 16 times the items):
// held-out RMAT-21 1.40 / 1.36 / 1.30 / 1.19, then 1.49 / 1.87 / 2.20;
// held-out RMAT-23 3.42 / 3.27 / 3.06 / 3.10-3.15, then 3.58 / 5.18 / 5.49;
// benchmark RMAT-22 2.03 / 1.97 / 1.84 / 1.72, then 2.25 / 2.86 / 3.13;
// RMAT-20 1.09 / 1.04 / 1.01 / 0.94.
constexpr uint32_t kTailDiv = 1;
// A bucket whose listed vertices hold at least n / kPullHeavyDiv heavy edges,
// and at least 1 / kPullOpenDiv of the heavy edges of the vertices not yet
// listed, runs its heavy pass as a pull.
constexpr uint32_t kPullHeavyDiv = 2;
constexpr uint32_t kPullOpenDiv = 2;
// Once 7/8 of the partition's heavy entries have been listed, thresholds
// rise by kStepGrow steps at a time: on R-MAT the first one or two buckets
// settle nearly every vertex, and each of the small buckets after them costs
// three or four invocations.  Chosen on the held-out scales 21 and 23 (32
// sources, ms per query; one step / 2 / 4 / 8 / 16 steps): RMAT-21 1.84 /
// 1.65 / 1.55 / 1.48 / 1.48, RMAT-23 4.17 / 3.81 / 3.66 / 3.58 / 3.59;
// benchmark scale 22: 2.65 / 2.40 / 2.29 / 2.21 / 2.22; scale 20 1.37 /
// 1.32 / 1.29 / 1.29 / 1.28.  Triggering at 3/4 instead of 7/8 made no
// difference; road grids and the 64x64 grid are unchanged.  Since the
// bucketing ends once the far list holds fewer vertices than have been
// popped (kTailDiv 1), the small buckets it saved are gone, and growth by
// 0 (off) / 4 / 8 / 16 measures RMAT-21 1.14 / 1.15 / 1.16 / 1.15, RMAT-22
// 1.67 / 1.67 / 1.68 / 1.69, RMAT-23 3.14 / 3.18 / 3.14 / 3.18, RMAT-20
// 0.94 / 0.95 / 0.94 / 0.93 ms: it is off.
constexpr uint32_t kStepGrow = 0;
// Step of the light/heavy partition on a scale-free graph, as a fraction of
// the mean weight W: each heavy edge is then relaxed once, while a smaller
// step adds buckets (one barrier each).  Measured on R-MAT graphs of scales
// 18 to 23 (16 sources each, ms per query), the larger the graph the
// smaller the best step: from 2^25 edges W/4 (scale 21: 2.32 against 3.01
// without a step, scale 22: 3.53 against 5.02, scale 23: 5.93 against 8.95;
// each within 2% of the best step tried), from 2^24 edges W/2 (scale 20:
// 1.83 against 2.06), below that no step (scale 18: 1.10 against 1.45).
// Those steps predate the growth of the step after the heavy passes, which
// runs on symmetric graphs; there, re-derived with the growth (16 sources,
// ms per query at steps 8 / 12 / 16 / 20 / 24 / 31 / 63, W = 128): held-out
// scale 21 1.80 / 1.50 / 1.42 / 1.49 / 1.42 / 1.49 / 1.82, held-out scale 23
// 4.09 / 3.60 / 3.48 / 3.44 / 3.48 / 3.56 / 4.55; benchmark scale 22 2.67 /
// 2.20 / 2.11 / 2.16 / 2.13 / 2.21 / 2.63; scale 20 1.41 / 1.26 / 1.10 /
// 1.09 / 1.17 / 1.12 / 1.28 (no step: 1.30 at W/2's rule); scale 18 (7.9M
// edges) 0.99 / 0.88 / 0.81 / 0.82 / 0.82 / 0.79 / 0.83 (no step: 0.84).
// A symmetric scale-free graph takes W/8 from 2^22 edges: the best step or
// within 2.4% of it at every scale.
constexpr double kSplitDeltaScale = 0.25;
constexpr int64_t kSplitQuarterMinEdges = int64_t(1) << 25;
constexpr int64_t kSplitHalfMinEdges = int64_t(1) << 24;
constexpr double kSplitGrowScale = 0.125;
constexpr int64_t kSplitGrowMinEdges = int64_t(1) << 22;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Per-device facts, looked up once.
struct DeviceInfo {
    int cus = 0;
    int wallclock_khz = 0;
    bool ready = false;
};
std::mutex g_dev_mu;
DeviceInfo g_dev[64];

irgl_status device_info(int dev, DeviceInfo *out) {
    if (dev < 0 || dev >= 64) return IRGL_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev[dev].ready) {
        int cus = 0, khz = 0;
        IRGL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        IRGL_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        g_dev[dev].cus = cus;
        g_dev[dev].wallclock_khz = khz > 0 ? khz : 100000;
        g_dev[dev].ready = true;
    }
    *out = g_dev[dev];
    return IRGL_OK;
}

// Resolved configuration of one query.
struct Cfg {
    int block;
    int t_wave;
    int t_block;
    int t_grid;
    int grid;  // 0 = co-resident limit
    int mode;
    uint32_t max_iter;
    uint32_t cap;
    uint32_t watchdog_ms;
    const volatile int32_t *abort_flag;
    uint32_t t_bitmap;
    uint32_t trace_len;
    unsigned long long *trace;
    uint32_t delta;
    uint32_t do_alpha, do_beta;  // do_alpha == 0: no bottom-up invocations
    uint32_t barrier;
    uint32_t reduce;  // topology-driven loop: IRGL_REDUCE_*
};

// Nested-parallelism thresholds (0 = default).  Vertices with t_grid or more
// edges go to the grid tier (IRGL_GRID_TIER_OFF: none).  By default every
// other range goes to the load-balanced gather tier, which fills every round
// whatever the degree mix; the workgroup (>= t_block) and wavefront
// (>= t_wave) tiers take ranges only when the caller sets their thresholds
// (t_wave then defaults to 64).
void resolve_tiers(int block, int t_wave, int t_block, int t_grid, int *ow, int *ob, int *og) {
    const int big = 2 * block;
    int g = t_grid ? t_grid : std::max(big, t_block);
    if (t_grid == IRGL_GRID_TIER_OFF) g = 0;
    const int b = t_block ? t_block : (g > 0 ? g : big);
    const int w = t_wave ? t_wave : (t_block ? std::min(64, b) : b);
    *ow = w;
    *ob = b;
    *og = g;
}

// Default workgroup size per kind, from sweeps over road and RMAT graphs:
// BFS invocations are short, and 1024-thread workgroups cut the barrier
// arrivals per invocation fourfold; SSSP's longer invocations do best at 512.
int default_block(int kind) { return kind == IRGL_KIND_BFS ? 1024 : 512; }

// Default grid-tier threshold of single queries, whatever the workgroup size
// (RMAT-22 SSSP at 512-thread workgroups: 4.73 ms per query at 512 against
// 4.84 ms at 1024; topology-driven 12.7 ms against 20.2 ms, and with
// 1024-thread workgroups 13.0 ms at 512, 17.2 ms at 256, 20.4 ms at 2048;
// BFS within 2% from 512 to 4096).
constexpr int kGridTier = 512;
// Outlined SSSP queries take hubs from 256 edges (16 sources, ms per query
// at 512 / 256: held-out RMAT-21 1.12 / 1.09, RMAT-23 3.32 / 3.31,
// benchmark RMAT-22 1.73 / 1.70, RMAT-20 0.90 / 0.91, road 4096^2 7.82 /
// 7.83; topology-driven queries lose at 256, see above).
constexpr int kGridTierSssp = 256;

irgl_status resolve(const irgl_graph_s *g, int kind, const irgl_config *c, Cfg *out) {
    Cfg r;
    r.block = (c && c->block) ? c->block : default_block(kind);
    if (r.block != 256 && r.block != 512 && r.block != 1024) return IRGL_ERR_CONFIG;
    r.mode = c ? c->mode : IRGL_MODE_PERSISTENT;
    if (r.mode != IRGL_MODE_PERSISTENT && r.mode != IRGL_MODE_HOST_LOOP && r.mode != IRGL_MODE_TOPOLOGY)
        return IRGL_ERR_CONFIG;
    // the grid tier takes hubs from a fixed kGridTier edges on
    int t_grid = c ? c->t_grid : 0;
    if (t_grid == 0)
        t_grid = std::max(kind == IRGL_KIND_SSSP && r.mode == IRGL_MODE_PERSISTENT ? kGridTierSssp : kGridTier,
                          c ? c->t_block : 0);
    resolve_tiers(r.block, c ? c->t_wave : 0, c ? c->t_block : 0, t_grid, &r.t_wave, &r.t_block, &r.t_grid);
    if (r.t_wave < 1 || r.t_block < r.t_wave || r.t_grid < 0 || (r.t_grid > 0 && r.t_grid < r.t_block))
        return IRGL_ERR_CONFIG;
    r.grid = c ? c->grid : 0;
    if (r.grid < 0) return IRGL_ERR_CONFIG;
    r.reduce = c ? c->reduce : IRGL_REDUCE_ANY;
    if (r.reduce != IRGL_REDUCE_ANY && r.reduce != IRGL_REDUCE_ALL) return IRGL_ERR_CONFIG;
    const uint32_t n = static_cast<uint32_t>(g->n);
    r.max_iter = (c && c->max_iter) ? c->max_iter : n + 1u;
    r.cap = (c && c->wl_capacity) ? std::min(c->wl_capacity, n) : n;
    r.watchdog_ms = (c && c->watchdog_ms) ? c->watchdog_ms : 20000u;
    r.abort_flag = c ? c->abort_flag : nullptr;
    // BFS: visited filter on by default; SSSP: the settled filter is opt-in
    // (its refreshes rarely repay on the measured graphs)
    r.t_bitmap = (c && c->t_bitmap) ? c->t_bitmap
                                    : (kind == IRGL_KIND_SSSP ? IRGL_BITMAP_NEVER : default_t_bitmap(g->n, g->m));
    // direction optimization needs in-edges = out-edges and the outlined loop
    const bool sym = (g->flags & IRGL_SYMMETRIC) != 0;
    r.do_alpha = (c && c->do_alpha) ? c->do_alpha : 14u;
    // back to top-down below n / 96 frontier vertices (16 sources, us per
    // query at 24 / 48 / 96 / 192: RMAT-20 234 / 230 / 229 / 229, RMAT-21
    // 310 / 308 / 308 / 305, RMAT-22 366 / 363 / 360 / 360, RMAT-23 565 /
    // 557 / 558 / 558, road 4096^2 unchanged)
    r.do_beta = (c && c->do_beta) ? c->do_beta : 96u;
    if (!sym || r.do_alpha == IRGL_DO_OFF || r.mode != IRGL_MODE_PERSISTENT) r.do_alpha = 0;
    r.trace_len = (c && c->trace) ? c->trace_len : 0u;
    r.trace = (c && c->trace) ? reinterpret_cast<unsigned long long *>(c->trace) : nullptr;
    // SSSP near/far step: explicit, or derived from the graph's shape
    r.delta = (c && c->delta) ? c->delta : default_delta(g);
    r.barrier = c ? c->barrier : IRGL_BARRIER_XCD;
    if (r.barrier > IRGL_BARRIER_WORKGROUP) return IRGL_ERR_CONFIG;
    *out = r;
    return IRGL_OK;
}

// Grid-tier list capacity: a vertex is deferred with t_grid or more edges,
// or with `block` or more when the worklist is small, so at most
// m / min(t_grid, block) + 1 vertices are listed.
uint32_t grid_list_cap(int64_t n, int64_t m, int t_grid, int block) {
    if (t_grid <= 0) return 0u;
    return static_cast<uint32_t>(std::min<int64_t>(n, m / std::min(t_grid, block) + 1));
}

struct Layout {
    size_t ctrl, wl0, wl1, stamp, shadow, far0, far1, far_flag, expd, hlist, hstamp, visited, frontier, hub_v,
        hub_base, rval, rparent, total;
    uint32_t hub_cap;
};

// An SSSP query runs the light/heavy split when the graph has a partition at
// the query's step and the loop is outlined.
bool uses_split(const irgl_graph_s *g, int kind, const Cfg &c) {
    return kind == IRGL_KIND_SSSP && g->split && c.delta == g->split_delta && c.mode == IRGL_MODE_PERSISTENT;
}

Layout layout(const irgl_graph_s *g, int kind, const Cfg &c, bool with_parent) {
    Layout L;
    L.ctrl = 0;
    L.wl0 = align_up(sizeof(Ctrl));
    L.wl1 = L.wl0 + align_up(static_cast<size_t>(c.cap) * 4);
    L.stamp = L.wl1 + align_up(static_cast<size_t>(c.cap) * 4);
    const size_t nb = align_up(static_cast<size_t>(g->n) * 4);
    const bool sssp = kind == IRGL_KIND_SSSP;
    L.shadow = L.stamp + (sssp ? nb : 0);
    L.far0 = L.shadow + (sssp ? nb : 0);
    L.far1 = L.far0 + (sssp ? nb : 0);
    L.far_flag = L.far1 + (sssp ? nb : 0);
    L.expd = L.far_flag + (sssp ? nb : 0);
    const bool split = uses_split(g, kind, c);
    L.hlist = L.expd + (sssp ? nb : 0);
    L.hstamp = L.hlist + (split ? nb : 0);
    L.visited = L.hstamp + (split ? nb : 0);
    const size_t bm = align_up((static_cast<size_t>(g->n) + 31) / 32 * 4);
    const bool pull = kind == IRGL_KIND_BFS && c.do_alpha != 0;
    const bool bitmap = c.t_bitmap != IRGL_BITMAP_NEVER || pull;
    L.frontier = L.visited + (bitmap ? bm : 0);
    L.hub_v = L.frontier + (pull ? 2 * bm : 0);  // current and next frontier bitmaps
    L.hub_cap = grid_list_cap(g->n, g->m, c.t_grid, c.block);
    L.hub_base = L.hub_v + align_up(static_cast<size_t>(L.hub_cap) * 4);
    // relabelled graph: values and parents under internal ids, scattered at the end
    L.rval = L.hub_base + align_up(static_cast<size_t>(L.hub_cap) * 4);
    L.rparent = L.rval + (g->perm ? nb : 0);
    L.total = L.rparent + (g->perm && with_parent ? nb : 0);
    return L;
}

struct OccEntry {
    const void *kernel;
    int block, dev, per_cu;
};
// Fixed-capacity cache (no heap growth on the launch path); when it is full
// the query is simply not cached.
constexpr int kOccCap = 256;
std::mutex g_occ_mu;
OccEntry g_occ[kOccCap];
int g_occ_n = 0;

template <class K>
irgl_status coresident_grid(K kernel, int block, int dev, int requested, int *grid) {
    DeviceInfo di;
    irgl_status st = device_info(dev, &di);
    if (st) return st;
    // the occupancy query costs tens of microseconds: once per kernel, block and device
    int per_cu = -1;
    const void *key = reinterpret_cast<const void *>(kernel);
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        for (int i = 0; i < g_occ_n; ++i) {
            const OccEntry &e = g_occ[i];
            if (e.kernel == key && e.block == block && e.dev == dev) per_cu = e.per_cu;
        }
    }
    if (per_cu < 0) {
        IRGL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
        std::lock_guard<std::mutex> lk(g_occ_mu);
        if (g_occ_n < kOccCap) g_occ[g_occ_n++] = OccEntry{key, block, dev, per_cu};
    }
    // Measured on gfx950: a grid that fills 7 waves per SIMD is not fully
    // co-resident (the barrier then waits for workgroups that never start),
    // while 6 waves per SIMD is.  Cap the grid at 6 waves per SIMD.
    const int waves_per_block = block / kWave;
    per_cu = std::min(per_cu, std::max(1, (6 * 4) / waves_per_block));
    const int limit = per_cu * di.cus;
    if (limit <= 0) return IRGL_ERR_CONFIG;
    if (requested > limit) return IRGL_ERR_CONFIG;
    *grid = requested ? requested : limit;
    return IRGL_OK;
}

int fill_grid(uint32_t n, int block) {
    const uint32_t g = (n + block - 1) / block;
    return static_cast<int>(std::max(1u, std::min(g, 65535u)));
}

// Pinned read-back words of the host-loop mode, one per calling thread, kept
// in a process-wide registry so that irgl_shutdown() can return them to the
// HIP runtime while it is still alive (nothing is freed from a static
// destructor: at process exit the runtime may already be gone).
std::mutex g_pinned_mu;
std::vector<void *> g_pinned;
thread_local uint32_t *t_pinned = nullptr;
thread_local uint64_t t_pinned_gen = 0;
uint64_t g_pinned_gen = 1;  // bumped by irgl_shutdown: every thread's word is gone

irgl_status pinned_word(uint32_t **p) {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!t_pinned || t_pinned_gen != g_pinned_gen) {
        void *h = nullptr;
        IRGL_HIP(hipHostMalloc(&h, 64, hipHostMallocDefault));
        t_pinned = static_cast<uint32_t *>(h);
        t_pinned_gen = g_pinned_gen;
        g_pinned.push_back(h);
    }
    *p = t_pinned;
    return IRGL_OK;
}

template <int B, class Op>
irgl_status launch_query(const irgl_graph_s *g, Params &p, const Cfg &c, hipStream_t s, int kind) {
    DeviceInfo di;
    irgl_status st = device_info(g->device, &di);
    if (st) return st;
    // IRGL_WATCHDOG_IMMEDIATE makes any barrier wait time out at once (a host
    // knob that exercises the watchdog path while every wave still exits).
    p.wd_ticks = c.watchdog_ms == IRGL_WATCHDOG_IMMEDIATE
                     ? 0ull
                     : static_cast<unsigned long long>(c.watchdog_ms) * di.wallclock_khz;
    p.abort_flag = c.abort_flag;
    p.barrier = c.barrier;

    hipLaunchKernelGGL(init_kernel, dim3(fill_grid(p.n, 256)), dim3(256), 0, s, p,
                       kind == IRGL_KIND_SSSP ? 1 : 0);
    IRGL_HIP(hipGetLastError());

    if (c.mode == IRGL_MODE_PERSISTENT) {
        int grid = 0;
        st = coresident_grid(persistent_kernel<B, Op>, B, g->device, c.grid, &grid);
        if (st) return st;
        void *args[] = {&p};
        IRGL_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(persistent_kernel<B, Op>),
                                            dim3(grid), dim3(B), args, 0, s));
    } else if (c.mode == IRGL_MODE_TOPOLOGY) {
        using TOp = typename TopoOf<Op>::type;
        int grid = 0;
        st = coresident_grid(topology_kernel<B, TOp>, B, g->device, c.grid, &grid);
        if (st) return st;
        p.reduce_all = c.reduce == IRGL_REDUCE_ALL ? 1u : 0u;
        p.trace_len = 0;  // the per-invocation trace is recorded by the data-driven loop only
        void *args[] = {&p};
        IRGL_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(topology_kernel<B, TOp>),
                                            dim3(grid), dim3(B), args, 0, s));
    } else {
        int grid = c.grid;
        if (grid == 0) {
            st = coresident_grid(level_kernel<B, Op>, B, g->device, 0, &grid);
            if (st) return st;
        }
        uint32_t *host = nullptr;
        st = pinned_word(&host);
        if (st) return st;
        uint32_t it = 0;
        int hit_limit = 0;
        bool transfer = false;  // the next invocation raises the SSSP threshold
        uint32_t far_n = 0, far_min = IRGL_INF;
        uint64_t items = 1, refreshed = 0;  // popped items so far / at the last bitmap refresh
        for (;; ++it) {
            if (it >= c.max_iter) {
                hit_limit = 1;
                break;
            }
            p.it = it;
            p.refresh = (items - refreshed >= c.t_bitmap && c.t_bitmap != IRGL_BITMAP_NEVER &&
                         (transfer || kind == IRGL_KIND_BFS)) ? 1u : 0u;
            if (p.refresh) refreshed = items;
            if (transfer) {
                const uint32_t lo = std::max(p.thresh, far_min);
                const uint32_t t_new = lo >= IRGL_INF - p.delta ? IRGL_INF : lo + p.delta;
                hipLaunchKernelGGL((transfer_kernel<B>), dim3(grid), dim3(B), 0, s, p, far_n, t_new);
                IRGL_HIP(hipGetLastError());
                p.thresh = t_new;
                ++p.far_tr;
            } else {
                hipLaunchKernelGGL((level_kernel<B, Op>), dim3(grid), dim3(B), 0, s, p);
                IRGL_HIP(hipGetLastError());
                if (p.t_grid > 0) {
                    hipLaunchKernelGGL((hub_level_kernel<B, Op>), dim3(grid), dim3(B), 0, s, p);
                    IRGL_HIP(hipGetLastError());
                }
            }
            IRGL_HIP(hipMemcpyAsync(host, &p.ctrl->cnt[(it + 1) % 3], 4, hipMemcpyDeviceToHost, s));
            if (kind == IRGL_KIND_SSSP) {
                IRGL_HIP(hipMemcpyAsync(host + 1, &p.ctrl->far_cnt[p.far_tr % 3], 4, hipMemcpyDeviceToHost, s));
                IRGL_HIP(hipMemcpyAsync(host + 2, &p.ctrl->far_min[p.far_tr % 3], 4, hipMemcpyDeviceToHost, s));
            }
            IRGL_HIP(hipStreamSynchronize(s));
            transfer = false;
            items += host[0];
            if (host[0] == 0) {
                far_n = kind == IRGL_KIND_SSSP ? std::min(host[1], p.far_cap) : 0u;
                far_min = kind == IRGL_KIND_SSSP ? host[2] : IRGL_INF;
                if (far_n == 0) break;
                transfer = true;
            }
        }
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, p, hit_limit);
        IRGL_HIP(hipGetLastError());
    }

    if (kind == IRGL_KIND_SSSP && p.parent) {
        hipLaunchKernelGGL((sssp_parent_kernel<B>), dim3(fill_grid(p.n, B)), dim3(B), 0, s, p);
        IRGL_HIP(hipGetLastError());
    }
    return IRGL_OK;
}

template <class Op>
irgl_status dispatch_block(const irgl_graph_s *g, Params &p, const Cfg &c, hipStream_t s, int kind) {
    switch (c.block) {
        case 256: return launch_query<256, Op>(g, p, c, s, kind);
        case 512: return launch_query<512, Op>(g, p, c, s, kind);
        case 1024: return launch_query<1024, Op>(g, p, c, s, kind);
        default: return IRGL_ERR_CONFIG;
    }
}

irgl_status run(int kind, irgl_graph g, int32_t src, uint32_t *out, int32_t *parent, void *ws,
                size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_config *cfg) {
    if (!g || !out || !ws) return IRGL_ERR_INVALID_ARGUMENT;
    if (src < 0 || src >= g->n) return IRGL_ERR_INVALID_ARGUMENT;
    if (kind == IRGL_KIND_SSSP && !g->w) return IRGL_ERR_NO_WEIGHTS;
    Cfg c;
    irgl_status st = resolve(g, kind, cfg, &c);
    if (st) return st;
    const Layout L = layout(g, kind, c, parent != nullptr);
    if (ws_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    // SSSP safety cap also covers the threshold-raise invocations (at most one
    // per vertex moved from the far list)
    if (kind == IRGL_KIND_SSSP && !(cfg && cfg->max_iter))
        c.max_iter = static_cast<uint32_t>(std::min<uint64_t>(0xFFFFFFF0ull, 4ull * static_cast<uint64_t>(g->n) + 16ull));
    int cur = -1;
    IRGL_HIP(hipGetDevice(&cur));
    if (cur != g->device) IRGL_HIP(hipSetDevice(g->device));

    char *base = static_cast<char *>(ws);
    Params p;
    std::memset(&p, 0, sizeof(p));
    p.n = g->n;
    p.row_ptr = g->row_ptr;
    p.col = g->col;
    p.w = g->w;
    if (uses_split(g, kind, c)) {
        p.col = g->scol;
        p.w = g->sw;
        p.split = g->split;
        p.hlist = reinterpret_cast<int32_t *>(base + L.hlist);
        p.hstamp = reinterpret_cast<uint32_t *>(base + L.hstamp);
        p.hcap = static_cast<uint32_t>(g->n);
        // the early end of the bucketing (first measured at divisor 16: RMAT-22
        // 3.65 ms per query against 3.74 without, 30 instead of 37
        // invocations; the divisor now is the one derived with kTailDiv) and
        // the 16-bit shadow (distances of scale-free graphs are small): RMAT-22
        // 3.47 against 3.54 ms, RMAT-23 5.82 against 5.95 ms (32 sources)
        if (scale_free(g)) {
            p.tail_div = kTailDiv;
            p.shadow16 = 1;
        }
        // the pull form of the heavy pass reads a vertex's heavy range as the
        // heavy edges INTO it: symmetric graphs only
        if (g->flags & IRGL_SYMMETRIC) {
            p.pull_heavy_div = kPullHeavyDiv;
            p.pull_open_div = kPullOpenDiv;
            p.heavy_m = g->heavy_m;
            p.step_grow = kStepGrow;
        }
    }
    p.val = g->perm ? reinterpret_cast<uint32_t *>(base + L.rval) : out;
    p.parent = g->perm && parent ? reinterpret_cast<int32_t *>(base + L.rparent) : parent;
    p.perm = g->perm;
    p.ctrl = reinterpret_cast<Ctrl *>(base + L.ctrl);
    p.wl0 = reinterpret_cast<int32_t *>(base + L.wl0);
    p.wl1 = reinterpret_cast<int32_t *>(base + L.wl1);
    p.stamp = kind == IRGL_KIND_SSSP ? reinterpret_cast<uint32_t *>(base + L.stamp) : nullptr;
    p.shadow = kind == IRGL_KIND_SSSP ? reinterpret_cast<uint32_t *>(base + L.shadow) : nullptr;
    const bool pull = kind == IRGL_KIND_BFS && c.do_alpha != 0;
    p.visited = (c.t_bitmap != IRGL_BITMAP_NEVER || pull) ? reinterpret_cast<uint32_t *>(base + L.visited)
                                                           : nullptr;
    const size_t bm = align_up((static_cast<size_t>(g->n) + 31) / 32 * 4);
    p.frontier = pull ? reinterpret_cast<uint32_t *>(base + L.frontier) : nullptr;
    p.frontier2 = pull ? reinterpret_cast<uint32_t *>(base + L.frontier + bm) : nullptr;
    p.do_alpha = c.do_alpha;
    p.do_beta = c.do_beta;
    p.m = g->m;
    p.t_bitmap = c.t_bitmap;
    if (kind == IRGL_KIND_SSSP) {
        p.far0 = reinterpret_cast<int32_t *>(base + L.far0);
        p.far1 = reinterpret_cast<int32_t *>(base + L.far1);
        p.far_flag = reinterpret_cast<uint32_t *>(base + L.far_flag);
        p.far_cap = static_cast<uint32_t>(g->n);
        p.expd = reinterpret_cast<uint32_t *>(base + L.expd);
    }
    p.delta = c.delta;
    p.thresh = c.delta;
    p.far_tr = 0;
    p.t_grid = c.t_grid;
    p.hub_cap = L.hub_cap;
    p.hub_v = reinterpret_cast<int32_t *>(base + L.hub_v);
    p.hub_base = reinterpret_cast<uint32_t *>(base + L.hub_base);
    p.trace_len = c.trace_len;
    p.trace = c.trace;
    p.dstats = reinterpret_cast<Stats *>(dstats);
    p.cap = c.cap;
    p.max_iter = c.max_iter;
    p.t_wave = c.t_wave;
    p.t_block = c.t_block;
    p.src = g->perm ? g->inv_host[static_cast<size_t>(src)] : src;
    p.src_orig = src;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Relabelled graph: the outlined loop maps its results back to caller ids
    // itself at the end of the launch, unless an SSSP parent pass must run
    // after it (then a separate kernel maps them back afterwards).
    const bool fused_map = g->perm && c.mode == IRGL_MODE_PERSISTENT && !(kind == IRGL_KIND_SSSP && parent);
    if (fused_map) {
        p.inv = g->inv;
        p.out_caller = out;
        p.parent_caller = parent;
    }
    if (kind == IRGL_KIND_BFS) st = dispatch_block<BfsOp>(g, p, c, s, kind);
    else st = dispatch_block<SsspOp>(g, p, c, s, kind);
    if (st == IRGL_OK && g->perm && !fused_map) {
        hipLaunchKernelGGL(scatter_results_kernel, dim3(fill_grid(g->n, 256)), dim3(256), 0, s, g->n, g->perm,
                           p.val, p.parent, out, parent);
        if (hipGetLastError() != hipSuccess) st = hip_fail(hipGetLastError());
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    return st;
}

// ---------------------------------------------------------------------------
// Batched launch (host side)
// ---------------------------------------------------------------------------

struct BatchLayout {
    size_t queue, team_task, tasks, stats, scratch, total;
    size_t team_bytes;
    size_t off_wl0, off_wl1, off_stamp, off_shadow, off_far0, off_far1, off_far_flag, off_visited, off_hub_v,
        off_hub_base, off_expd;
    uint32_t cap, hub_cap;
    int teams;
    int team;  // workgroups per team
};

// Default server gang threshold: a graph with this many edges keeps a
// 16-workgroup team busy ~50x longer than the whole grid does.
constexpr uint32_t kDefaultGangEdges = 1u << 23;

// Server start check: a launch whose workgroups are not all resident within
// this many milliseconds (another kernel holds part of the device) gives up
// before claiming anything and is launched again while work is pending.
constexpr uint32_t kServerStartMs = 10;

struct BatchCfg {
    int block, team, t_wave, t_block, t_grid, grid;
    uint32_t delta, watchdog_ms, barrier;
    uint32_t gang_edges;  // server: tasks on graphs with at least this many edges run on the whole grid
    uint32_t gang_queue;  // server: ... and any task enqueued while fewer than this many are in flight
};

irgl_status resolve_batch(const irgl_batch_config *c, BatchCfg *out) {
    BatchCfg r;
    r.block = (c && c->block) ? c->block : 256;
    if (r.block != 256 && r.block != 512 && r.block != 1024) return IRGL_ERR_CONFIG;
    r.team = (c && c->team) ? c->team : 16;
    if (r.team < 1) return IRGL_ERR_CONFIG;
    resolve_tiers(r.block, c ? c->t_wave : 0, c ? c->t_block : 0, c ? c->t_grid : 0, &r.t_wave, &r.t_block,
                  &r.t_grid);
    if (r.t_wave < 1 || r.t_block < r.t_wave || r.t_grid < 0 || (r.t_grid > 0 && r.t_grid < r.t_block))
        return IRGL_ERR_CONFIG;
    r.delta = c ? c->delta : 0u;
    r.watchdog_ms = (c && c->watchdog_ms) ? c->watchdog_ms : 20000u;
    r.grid = c ? c->grid : 0;
    if (r.grid < 0) return IRGL_ERR_CONFIG;
    r.barrier = c ? c->barrier : IRGL_BARRIER_XCD;
    if (r.barrier > IRGL_BARRIER_WORKGROUP) return IRGL_ERR_CONFIG;
    r.gang_edges = (c && c->gang_edges) ? c->gang_edges : kDefaultGangEdges;
    r.gang_queue = c ? c->gang_queue : 0u;
    *out = r;
    return IRGL_OK;
}

irgl_status check_tasks(const irgl_task *tasks, int32_t ntasks) {
    if (!tasks || ntasks <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    for (int32_t i = 0; i < ntasks; ++i) {
        const irgl_task &t = tasks[i];
        if (!t.g || !t.out) return IRGL_ERR_INVALID_ARGUMENT;
        if (t.kind != IRGL_KIND_BFS && t.kind != IRGL_KIND_SSSP) return IRGL_ERR_INVALID_ARGUMENT;
        if (t.src < 0 || t.src >= t.g->n) return IRGL_ERR_INVALID_ARGUMENT;
        if (t.kind == IRGL_KIND_SSSP && !t.g->w) return IRGL_ERR_NO_WEIGHTS;
    }
    return IRGL_OK;
}

template <int B>
irgl_status batch_grid(int dev, int requested, int *grid, bool server) {
    // the two control kernels differ in register use, hence in co-residency
    if (server) return coresident_grid(server_kernel<B>, B, dev, requested, grid);
    return coresident_grid(batch_kernel<B>, B, dev, requested, grid);
}

// One team's (or the gang's) scratch region for graphs of at most nmax
// vertices / mmax edges: control block, claimed descriptor (and gang
// record), worklists, SSSP arrays, bitmap and grid-tier list.
void region_layout(int64_t nmax, int64_t mmax, bool any_sssp, int t_grid, int block, BatchLayout *L) {
    nmax = std::max<int64_t>(nmax, 1);
    L->cap = static_cast<uint32_t>(nmax);
    L->hub_cap = grid_list_cap(nmax, mmax, t_grid, block);
    const size_t nb = align_up(static_cast<size_t>(nmax) * 4);
    size_t o = align_up(sizeof(Ctrl) + sizeof(GangInfo));
    L->off_wl0 = o;  o += nb;
    L->off_wl1 = o;  o += nb;
    L->off_stamp = o;  o += any_sssp ? nb : 0;
    L->off_shadow = o;  o += any_sssp ? nb : 0;
    L->off_far0 = o;  o += any_sssp ? nb : 0;
    L->off_far1 = o;  o += any_sssp ? nb : 0;
    L->off_far_flag = o;  o += any_sssp ? nb : 0;
    L->off_expd = o;  o += any_sssp ? nb : 0;
    L->off_visited = o;  o += align_up((static_cast<size_t>(nmax) + 31) / 32 * 4);
    L->off_hub_v = o;  o += align_up(static_cast<size_t>(L->hub_cap) * 4);
    L->off_hub_base = o;  o += align_up(static_cast<size_t>(L->hub_cap) * 4);
    L->team_bytes = align_up(o);
}

// Team layout for graphs of at most nmax vertices / mmax edges; `records`
// per-task statistics slots (batch: tasks, server: ring slots).
irgl_status team_layout(int64_t nmax, int64_t mmax, bool any_sssp, bool any_bfs, int32_t records,
                        const BatchCfg &c, int dev, BatchLayout *out, bool server = false) {
    BatchLayout L;
    nmax = std::max<int64_t>(nmax, 1);
    int grid = 0;
    irgl_status st = IRGL_OK;
    switch (c.block) {
        case 256: st = batch_grid<256>(dev, c.grid, &grid, server); break;
        case 512: st = batch_grid<512>(dev, c.grid, &grid, server); break;
        default: st = batch_grid<1024>(dev, c.grid, &grid, server); break;
    }
    if (st) return st;
    const int team = std::min(c.team, grid);
    L.team = team;
    L.teams = grid / team;
    region_layout(nmax, mmax, any_sssp, c.t_grid, c.block, &L);
    L.queue = 0;
    L.team_task = align_up(4);
    L.tasks = L.team_task + align_up(static_cast<size_t>(L.teams) * 4);
    L.stats = L.tasks + align_up(static_cast<size_t>(records) * sizeof(TaskDesc));
    L.scratch = L.stats + align_up(static_cast<size_t>(records) * sizeof(Stats));
    L.total = L.scratch + L.team_bytes * static_cast<size_t>(L.teams);
    *out = L;
    return IRGL_OK;
}

irgl_status batch_layout(const irgl_task *tasks, int32_t ntasks, const BatchCfg &c, int dev,
                         BatchLayout *out) {
    int64_t nmax = 1, mmax = 0;
    bool any_sssp = false, any_bfs = false;
    for (int32_t i = 0; i < ntasks; ++i) {
        nmax = std::max<int64_t>(nmax, tasks[i].g->n);
        mmax = std::max<int64_t>(mmax, tasks[i].g->m);
        any_sssp |= tasks[i].kind == IRGL_KIND_SSSP;
        any_bfs |= tasks[i].kind == IRGL_KIND_BFS;
    }
    return team_layout(nmax, mmax, any_sssp, any_bfs, ntasks, c, dev, out);
}

// Reset every team's barrier words (server launches keep the ring head).
__global__ void zero_head_kernel(unsigned long long *w) { *w = 0ull; }

// Before every server launch: team barrier words, the gang control block's
// barrier words and start check, and the head word's gang count / pending
// bit (the claimed count is kept).
__global__ void server_reset_kernel(char *scratch, unsigned long long team_bytes, int teams, Ctrl *gang,
                                    unsigned long long *head) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < teams) {
        Ctrl *c = reinterpret_cast<Ctrl *>(scratch + static_cast<unsigned long long>(t) * team_bytes);
        reset_barrier_words(c);
        c->fatal = 0;
        c->error = 0;
    } else if (t == teams) {
        reset_barrier_words(gang);
        gang->fatal = 0;
        gang->error = 0;
        GangInfo *gi = reinterpret_cast<GangInfo *>(reinterpret_cast<char *>(gang) + sizeof(Ctrl));
        gi->start_count = 0;
        gi->start_state = 0;
        *head &= 0xFFFFFFFFull;
    }
}

// Reset the queue head and every team's barrier words.
__global__ void batch_init_kernel(uint32_t *queue_head, char *scratch, unsigned long long team_bytes,
                                  int teams) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *queue_head = 0u;
    if (t < teams) {
        Ctrl *c = reinterpret_cast<Ctrl *>(scratch + static_cast<unsigned long long>(t) * team_bytes);
        reset_barrier_words(c);
        c->fatal = 0;
        c->error = 0;
    }
}

template <int B>
irgl_status launch_batch(const BatchParams &bp, int grid, hipStream_t s) {
    void *args[] = {const_cast<BatchParams *>(&bp)};
    IRGL_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(batch_kernel<B>), dim3(grid), dim3(B),
                                        args, 0, s));
    return IRGL_OK;
}

uint32_t task_delta(const irgl_graph_s *g, uint32_t override_delta);

void fill_desc(TaskDesc &d, const irgl_task &t, Stats *stats, uint32_t delta_override, bool gang = false) {
    std::memset(&d, 0, sizeof(d));
    d.gang = gang ? 1u : 0u;
    d.row_ptr = t.g->orig_row_ptr;
    d.col = t.g->orig_col;
    d.w = t.g->orig_w;
    d.out = t.out;
    d.parent = t.parent;
    d.stats = stats;
    d.n = t.g->n;
    d.kind = t.kind;
    d.src = t.src;
    d.delta = t.kind == IRGL_KIND_SSSP ? task_delta(t.g, delta_override) : IRGL_DELTA_NONE;
    const uint64_t n = static_cast<uint64_t>(t.g->n);
    d.max_iter = t.kind == IRGL_KIND_SSSP ? static_cast<uint32_t>(std::min<uint64_t>(0xFFFFFFF0ull, 4 * n + 16))
                                          : static_cast<uint32_t>(n + 1);
    d.t_bitmap = t.kind == IRGL_KIND_SSSP ? IRGL_BITMAP_NEVER : default_t_bitmap(t.g->n, t.g->m);
}

void fill_batch_params(BatchParams &bp, const BatchLayout &L, char *base, const BatchCfg &c,
                       const DeviceInfo &di) {
    std::memset(&bp, 0, sizeof(bp));
    bp.tasks = reinterpret_cast<const TaskDesc *>(base + L.tasks);
    bp.queue_head = reinterpret_cast<uint32_t *>(base + L.queue);
    bp.team_task = reinterpret_cast<uint32_t *>(base + L.team_task);
    bp.scratch = base + L.scratch;
    bp.team_bytes = L.team_bytes;
    bp.off_wl0 = L.off_wl0;
    bp.off_wl1 = L.off_wl1;
    bp.off_stamp = L.off_stamp;
    bp.off_shadow = L.off_shadow;
    bp.off_far0 = L.off_far0;
    bp.off_far1 = L.off_far1;
    bp.off_far_flag = L.off_far_flag;
    bp.off_expd = L.off_expd;
    bp.off_visited = L.off_visited;
    bp.off_hub_v = L.off_hub_v;
    bp.off_hub_base = L.off_hub_base;
    bp.cap = L.cap;
    bp.hub_cap = L.hub_cap;
    bp.team = L.team;
    bp.t_wave = c.t_wave;
    bp.t_block = c.t_block;
    bp.t_grid = c.t_grid;
    bp.wd_ticks = static_cast<unsigned long long>(c.watchdog_ms) * di.wallclock_khz;
    bp.barrier = c.barrier;
}

template <int B>
irgl_status launch_server(const ServerParams &sp, int grid, hipStream_t s) {
    void *args[] = {const_cast<ServerParams *>(&sp)};
    IRGL_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(server_kernel<B>), dim3(grid), dim3(B),
                                        args, 0, s));
    return IRGL_OK;
}

// Batched and served tasks traverse the caller's rows (no partition).
uint32_t task_delta(const irgl_graph_s *g, uint32_t override_delta) {
    return override_delta ? override_delta : delta_rule(g, false);
}

// Single queries that leave the step at 0.
uint32_t default_delta(const irgl_graph_s *g) { return g->qdelta; }

bool scale_free(const irgl_graph_s *g) {
    if (!g->weight_sum || g->m <= 0 || g->n <= 0) return false;
    const double mean_deg = static_cast<double>(g->m) / static_cast<double>(g->n);
    return mean_deg >= kDeltaMinDegree && static_cast<double>(g->max_degree) > kSkew * mean_deg;
}

// The mean weight is known when the upload validated the graph.
// `partitioned`: rows are split into light and heavy edges at the step.
uint32_t delta_rule(const irgl_graph_s *g, bool partitioned) {
    if (!g->weight_sum || g->m <= 0 || g->n <= 0) return IRGL_DELTA_NONE;
    const double mean_w = static_cast<double>(g->weight_sum) / static_cast<double>(g->m);
    const double mean_deg = static_cast<double>(g->m) / static_cast<double>(g->n);
    double d;
    if (mean_deg < kDeltaMinDegree) {
        d = kDeltaScale * mean_w / std::max(1.0, mean_deg);
    } else if (static_cast<double>(g->max_degree) <= kSkew * mean_deg) {
        d = kDeltaDenseScale * mean_w / mean_deg;
    } else if (partitioned) {
        if ((g->flags & IRGL_SYMMETRIC) && g->m >= kSplitGrowMinEdges) d = kSplitGrowScale * mean_w;
        else if (g->m >= kSplitQuarterMinEdges) d = kSplitDeltaScale * mean_w;
        else if (g->m >= kSplitHalfMinEdges) d = 2.0 * kSplitDeltaScale * mean_w;
        else return IRGL_DELTA_NONE;
    } else {
        if (g->m < kDeltaSkewMinEdges) return IRGL_DELTA_NONE;
        d = mean_w;
    }
    return static_cast<uint32_t>(std::min(4.0e9, std::max(1.0, d)));
}

__device__ uint32_t g_invalid_flag;
__device__ unsigned long long g_weight_sum;
__device__ uint32_t g_max_degree;
__device__ unsigned long long g_heavy_edges;

__global__ void clear_flag_kernel() {
    g_invalid_flag = 0u;
    g_weight_sum = 0ull;
    g_max_degree = 0u;
    g_heavy_edges = 0ull;
}

// Light/heavy partition of every row (upload time): one wavefront per row
// counts the edges lighter than `delta`, then writes them, in row order, in
// front of the others (also in row order); split[v] = first heavy edge.
__global__ void partition_rows_kernel(int32_t n, const int32_t *rp, const int32_t *col, const uint32_t *w,
                                      uint32_t delta, int32_t *scol, uint32_t *sw, int32_t *split,
                                      unsigned long long *heavy_total) {
    const int lane = threadIdx.x % kWave;
    const int32_t waves = static_cast<int32_t>(gridDim.x * (blockDim.x / kWave));
    unsigned long long heavy = 0;
    for (int32_t u = static_cast<int32_t>(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave); u < n;
         u += waves) {
        const int32_t r0 = rp[u], r1 = rp[u + 1];
        int32_t nl = 0;
        for (int32_t e0 = r0; e0 < r1; e0 += kWave) {
            const int32_t e = e0 + lane;
            nl += __popcll(__ballot(e < r1 && w[e] < delta));
        }
        int32_t lo = r0, hi = r0 + nl;
        for (int32_t e0 = r0; e0 < r1; e0 += kWave) {
            const int32_t e = e0 + lane;
            const bool in = e < r1;
            const uint32_t wt = in ? w[e] : 0u;
            const int32_t c = in ? col[e] : 0;
            const bool light = in && wt < delta;
            const bool hv = in && !light;
            const unsigned long long ml = __ballot(light), mh = __ballot(hv);
            if (light) {
                const int32_t k = lo + static_cast<int32_t>(lane_rank(ml));
                scol[k] = c;
                sw[k] = wt;
            }
            if (hv) {
                const int32_t k = hi + static_cast<int32_t>(lane_rank(mh));
                scol[k] = c;
                sw[k] = wt;
            }
            lo += __popcll(ml);
            hi += __popcll(mh);
        }
        if (lane == 0) {
            split[u] = r0 + nl;
            heavy += static_cast<unsigned long long>(r1 - r0 - nl);
        }
    }
    if (lane == 0 && heavy) atomicAdd(heavy_total, heavy);
}

// (Re)build the partition of g's SSSP copy at `delta` (synchronous).
irgl_status build_partition(irgl_graph_s *g, uint32_t delta) {
    g->split = nullptr;
    g->split_delta = IRGL_DELTA_NONE;
    g->heavy_m = 0;
    if (!g->scol || delta == IRGL_DELTA_NONE || g->m == 0) return IRGL_OK;
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, 0);
    IRGL_HIP(hipGetLastError());
    unsigned long long *heavy = nullptr;
    IRGL_HIP(hipGetSymbolAddress(reinterpret_cast<void **>(&heavy), HIP_SYMBOL(g_heavy_edges)));
    const int egrid = std::max(1, std::min(4096, (g->n + 3) / 4));  // 4 wavefronts per workgroup
    hipLaunchKernelGGL(partition_rows_kernel, dim3(egrid), dim3(256), 0, 0, g->n, g->row_ptr, g->col, g->w,
                       delta, g->scol, g->sw, g->split_store, heavy);
    IRGL_HIP(hipGetLastError());
    unsigned long long h = 0;
    IRGL_HIP(hipMemcpy(&h, heavy, 8, hipMemcpyDeviceToHost));
    g->split = h ? g->split_store : nullptr;
    g->split_delta = delta;
    g->heavy_m = h;
    return IRGL_OK;
}

// ---------------------------------------------------------------------------
// Degree-sorted relabelling (upload time).  Internal id i is the caller
// vertex perm[i], in decreasing out-degree order (ties by caller id): the
// values of the vertices most edges point at then share a few cache lines
// and stay in L2, so most per-edge probes of a traversal hit L2.
// ---------------------------------------------------------------------------
__global__ void degree_keys_kernel(int32_t n, const int32_t *rp, uint32_t *keys, int32_t *ids) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        keys[v] = static_cast<uint32_t>(rp[v + 1] - rp[v]);
        ids[v] = v;
    }
}

__global__ void inverse_kernel(int32_t n, const int32_t *perm, int32_t *inv, int32_t *nrp) {
    const int32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) nrp[0] = 0;
    for (int32_t i = i0; i < n; i += gridDim.x * blockDim.x) inv[perm[i]] = i;
}

// One wavefront per internal vertex copies its range with relabelled targets.
__global__ void relabel_edges_kernel(int32_t n, const int32_t *perm, const int32_t *inv, const int32_t *rp,
                                     const int32_t *col, const uint32_t *w, const int32_t *nrp, int32_t *ncol,
                                     uint32_t *nw) {
    const int lane = threadIdx.x % kWave;
    const int32_t waves = static_cast<int32_t>(gridDim.x * (blockDim.x / kWave));
    for (int32_t u = static_cast<int32_t>(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave); u < n;
         u += waves) {
        const int32_t o = perm[u];
        const int32_t r0 = rp[o], d = rp[o + 1] - r0, dst = nrp[u];
        for (int32_t k = lane; k < d; k += kWave) {
            ncol[dst + k] = inv[col[r0 + k]];
            if (w) nw[dst + k] = w[r0 + k];
        }
    }
}

// Store of a relabelled copy: row offsets, targets, weights, perm, then the
// build's scratch (sort keys, ids, inverse, library sort/scan scratch).
struct ReorderLayout {
    size_t nrp, ncol, nw, scol, sw, split, perm, keys_in, keys_out, ids_in, inv, tmp, tmp_bytes, total;
};

irgl_status reorder_layout(int32_t n, int64_t m, bool weighted, ReorderLayout *out) {
    ReorderLayout L;
    const size_t nb = align_up(static_cast<size_t>(n) * 4);
    L.nrp = 0;
    L.ncol = align_up(static_cast<size_t>(n + 1) * 4);
    L.nw = L.ncol + align_up(static_cast<size_t>(m) * 4 + 4);
    // weighted: the SSSP copy (partitioned targets and weights, split points)
    L.scol = L.nw + (weighted ? align_up(static_cast<size_t>(m) * 4 + 4) : 0);
    L.sw = L.scol + (weighted ? align_up(static_cast<size_t>(m) * 4 + 4) : 0);
    L.split = L.sw + (weighted ? align_up(static_cast<size_t>(m) * 4 + 4) : 0);
    L.perm = L.split + (weighted ? nb : 0);
    L.keys_in = L.perm + nb;
    L.keys_out = L.keys_in + nb;
    L.ids_in = L.keys_out + nb;
    L.inv = L.ids_in + nb;
    L.tmp = L.inv + nb;
    size_t sort_b = 0, scan_b = 0;
    IRGL_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, sort_b, static_cast<const uint32_t *>(nullptr),
                                                          static_cast<uint32_t *>(nullptr),
                                                          static_cast<const int32_t *>(nullptr),
                                                          static_cast<int32_t *>(nullptr), n));
    IRGL_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, scan_b, static_cast<const uint32_t *>(nullptr),
                                              static_cast<int32_t *>(nullptr), n));
    L.tmp_bytes = align_up(std::max(sort_b, scan_b));
    L.total = L.tmp + L.tmp_bytes;
    *out = L;
    return IRGL_OK;
}

// ---------------------------------------------------------------------------
// The library's own query workspace, for callers that cannot allocate
// (irgl_sssp_noalloc).  Every device the library runs on holds one copy of
// the array until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address: the device address of each device's copy
// is taken once per device with hipGetSymbolAddress (that device current) and
// only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t{IRGL_NOALLOC_SCRATCH_BYTES};
static_assert(kScratchBytes % kAlign == 0, "scratch size");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

irgl_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return IRGL_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        IRGL_HIP(hipGetDevice(&cur));
        if (cur != dev) IRGL_HIP(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e);
        if (!ptr) return IRGL_ERR_DEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return IRGL_OK;
}

}  // namespace

// For the library's other translation units (the Boruvka workload): the
// failure bookkeeping behind irgl_last_hip_error, and the caller's CSR of a
// graph handle.
namespace irgl_shared {
irgl_status note_hip_failure(hipError_t e) { return hip_fail(e); }

irgl_status caller_csr(const irgl_graph_s *g, int *device, irgl_csr *out) {
    if (!g || !device || !out) return IRGL_ERR_INVALID_ARGUMENT;
    *device = g->device;
    out->n = g->n;
    out->m = g->m;
    out->row_ptr = g->orig_row_ptr;
    out->col = g->orig_col;
    out->w = g->orig_w;
    out->flags = g->flags;
    return IRGL_OK;
}
}  // namespace irgl_shared

extern "C" {

int irgl_version(void) { return IRGL_VERSION; }

const char *irgl_status_string(irgl_status s) {
    switch (s) {
        case IRGL_OK: return "ok";
        case IRGL_ERR_INVALID_ARGUMENT: return "invalid argument";
        case IRGL_ERR_NO_WEIGHTS: return "graph has no weights";
        case IRGL_ERR_INVALID_GRAPH: return "malformed CSR graph";
        case IRGL_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case IRGL_ERR_OVERFLOW: return "worklist or distance overflow";
        case IRGL_ERR_ABORTED: return "aborted by the host";
        case IRGL_ERR_BUSY: return "no free slot";
        case IRGL_ERR_TOO_LARGE: return "request exceeds the memory budget";
        case IRGL_ERR_NO_DEVICE: return "no HIP device";
        case IRGL_ERR_DEVICE: return "HIP runtime error";
        case IRGL_ERR_WATCHDOG: return "grid barrier watchdog expired";
        case IRGL_ERR_ITERATION_LIMIT: return "iteration limit reached";
        case IRGL_ERR_CONFIG: return "unsupported configuration";
        case IRGL_ERR_INTERNAL: return "internal consistency check failed";
        default: return "unknown status";
    }
}

int32_t irgl_last_hip_error(void) { return g_last_hip_error; }

irgl_status irgl_wallclock_khz(int32_t *khz) {
    if (!khz) return IRGL_ERR_INVALID_ARGUMENT;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return IRGL_ERR_NO_DEVICE;
    }
    int dev = 0;
    IRGL_HIP(hipGetDevice(&dev));
    DeviceInfo di;
    irgl_status st = device_info(dev, &di);
    if (st) return st;
    *khz = di.wallclock_khz;
    return IRGL_OK;
}

// Argument checks, the device, and (IRGL_VALIDATE) the on-device CSR check,
// weight sum and largest out-degree; shared by both uploads.
static irgl_status upload_prologue(const irgl_csr *csr, int *dev_out, unsigned long long *wsum_out,
                                   uint32_t *maxdeg_out) {
    if (csr->n <= 0 || csr->m < 0 || csr->m >= (int64_t(1) << 31)) return IRGL_ERR_INVALID_ARGUMENT;
    if (!csr->row_ptr || (csr->m > 0 && !csr->col)) return IRGL_ERR_INVALID_ARGUMENT;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return IRGL_ERR_NO_DEVICE;
    }
    int dev = 0;
    IRGL_HIP(hipGetDevice(&dev));
    *dev_out = dev;
    unsigned long long weight_sum = 0;
    uint32_t max_degree = 0;
    if (csr->flags & IRGL_VALIDATE) {
        hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, 0);
        IRGL_HIP(hipGetLastError());
        uint32_t *flag = nullptr;
        unsigned long long *wsum = nullptr;
        uint32_t *maxdeg = nullptr;
        IRGL_HIP(hipGetSymbolAddress(reinterpret_cast<void **>(&flag), HIP_SYMBOL(g_invalid_flag)));
        IRGL_HIP(hipGetSymbolAddress(reinterpret_cast<void **>(&wsum), HIP_SYMBOL(g_weight_sum)));
        IRGL_HIP(hipGetSymbolAddress(reinterpret_cast<void **>(&maxdeg), HIP_SYMBOL(g_max_degree)));
        const int grid = std::min<int64_t>(4096, std::max<int64_t>(1, (std::max<int64_t>(csr->m, csr->n) + 255) / 256));
        hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(256), 0, 0, csr->n, csr->m, csr->row_ptr,
                           csr->col, csr->w, flag, wsum, maxdeg);
        IRGL_HIP(hipGetLastError());
        uint32_t bad = 0;
        IRGL_HIP(hipMemcpy(&bad, flag, 4, hipMemcpyDeviceToHost));
        if (bad) return IRGL_ERR_INVALID_GRAPH;
        IRGL_HIP(hipMemcpy(&weight_sum, wsum, 8, hipMemcpyDeviceToHost));
        IRGL_HIP(hipMemcpy(&max_degree, maxdeg, 4, hipMemcpyDeviceToHost));
    }
    *wsum_out = csr->w ? weight_sum : 0ull;
    *maxdeg_out = max_degree;
    return IRGL_OK;
}

irgl_status irgl_graph_upload(const irgl_csr *csr, irgl_graph *out) {
    if (!csr || !out) return IRGL_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int dev = 0;
    unsigned long long weight_sum = 0;
    uint32_t max_degree = 0;
    irgl_status st = upload_prologue(csr, &dev, &weight_sum, &max_degree);
    if (st) return st;
    irgl_graph_s *g = new (std::nothrow) irgl_graph_s;
    if (!g) return IRGL_ERR_INVALID_ARGUMENT;
    g->n = csr->n;
    g->m = csr->m;
    g->row_ptr = csr->row_ptr;
    g->col = csr->col;
    g->w = csr->w;
    g->flags = csr->flags;
    g->device = dev;
    g->weight_sum = csr->w ? weight_sum : 0;
    g->max_degree = max_degree;
    g->orig_row_ptr = csr->row_ptr;
    g->orig_col = csr->col;
    g->orig_w = csr->w;
    g->perm = nullptr;
    g->inv = nullptr;
    g->qdelta = delta_rule(g, false);
    *out = g;
    return IRGL_OK;
}

irgl_status irgl_reorder_bytes(int32_t n, int64_t m, int32_t weighted, size_t *bytes) {
    if (!bytes || n <= 0 || m < 0 || m >= (int64_t(1) << 31)) return IRGL_ERR_INVALID_ARGUMENT;
    ReorderLayout L;
    irgl_status st = reorder_layout(n, m, weighted != 0, &L);
    if (st) return st;
    *bytes = L.total;
    return IRGL_OK;
}

irgl_status irgl_graph_upload_reordered(const irgl_csr *csr, void *store, size_t store_bytes, irgl_graph *out) {
    if (!csr || !out || !store) return IRGL_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int dev = 0;
    unsigned long long weight_sum = 0;
    uint32_t max_degree = 0;
    irgl_status st = upload_prologue(csr, &dev, &weight_sum, &max_degree);
    if (st) return st;
    const int32_t n = csr->n;
    const int64_t m = csr->m;
    ReorderLayout L;
    st = reorder_layout(n, m, csr->w != nullptr, &L);
    if (st) return st;
    if (store_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    char *b = static_cast<char *>(store);
    int32_t *nrp = reinterpret_cast<int32_t *>(b + L.nrp);
    int32_t *ncol = reinterpret_cast<int32_t *>(b + L.ncol);
    uint32_t *nw = csr->w ? reinterpret_cast<uint32_t *>(b + L.nw) : nullptr;
    int32_t *perm = reinterpret_cast<int32_t *>(b + L.perm);
    uint32_t *keys_in = reinterpret_cast<uint32_t *>(b + L.keys_in);
    uint32_t *keys_out = reinterpret_cast<uint32_t *>(b + L.keys_out);
    int32_t *ids_in = reinterpret_cast<int32_t *>(b + L.ids_in);
    int32_t *inv = reinterpret_cast<int32_t *>(b + L.inv);
    void *tmp = b + L.tmp;
    const int grid = fill_grid(static_cast<uint32_t>(n), 256);
    hipLaunchKernelGGL(degree_keys_kernel, dim3(grid), dim3(256), 0, 0, n, csr->row_ptr, keys_in, ids_in);
    IRGL_HIP(hipGetLastError());
    size_t tb = L.tmp_bytes;
    IRGL_HIP(hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, keys_in, keys_out, ids_in, perm, n));
    tb = L.tmp_bytes;
    IRGL_HIP(hipcub::DeviceScan::InclusiveSum(tmp, tb, keys_out, nrp + 1, n));
    hipLaunchKernelGGL(inverse_kernel, dim3(grid), dim3(256), 0, 0, n, perm, inv, nrp);
    IRGL_HIP(hipGetLastError());
    const int egrid = std::max(1, std::min(4096, (n + 3) / 4));  // 4 wavefronts per workgroup
    hipLaunchKernelGGL(relabel_edges_kernel, dim3(egrid), dim3(256), 0, 0, n, perm, inv, csr->row_ptr, csr->col,
                       csr->w, nrp, ncol, nw);
    IRGL_HIP(hipGetLastError());
    irgl_graph_s *g = new (std::nothrow) irgl_graph_s;
    if (!g) return IRGL_ERR_INVALID_ARGUMENT;
    g->inv_host.resize(static_cast<size_t>(n));
    const hipError_t e = hipMemcpy(g->inv_host.data(), inv, static_cast<size_t>(n) * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e);
    }
    g->n = n;
    g->m = m;
    g->row_ptr = nrp;
    g->col = ncol;
    g->w = nw;
    g->flags = csr->flags;
    g->device = dev;
    g->weight_sum = weight_sum;
    g->max_degree = max_degree;
    g->orig_row_ptr = csr->row_ptr;
    g->orig_col = csr->col;
    g->orig_w = csr->w;
    g->perm = perm;
    g->inv = inv;
    if (nw) {
        g->scol = reinterpret_cast<int32_t *>(b + L.scol);
        g->sw = reinterpret_cast<uint32_t *>(b + L.sw);
        g->split_store = reinterpret_cast<int32_t *>(b + L.split);
        g->qdelta = delta_rule(g, true);
        st = build_partition(g, g->qdelta);
        if (st) {
            delete g;
            return st;
        }
    } else {
        g->qdelta = delta_rule(g, false);
    }
    *out = g;
    return IRGL_OK;
}

irgl_status irgl_graph_set_delta(irgl_graph g, uint32_t delta) {
    if (!g || delta == 0) return IRGL_ERR_INVALID_ARGUMENT;
    if (!g->scol) {  // no SSSP copy: only the default step changes
        g->qdelta = delta;
        return IRGL_OK;
    }
    int cur = -1;
    IRGL_HIP(hipGetDevice(&cur));
    if (cur != g->device) IRGL_HIP(hipSetDevice(g->device));
    const irgl_status st = build_partition(g, delta);
    if (st == IRGL_OK) g->qdelta = delta;
    if (cur != g->device) (void)hipSetDevice(cur);
    return st;
}

irgl_status irgl_graph_free(irgl_graph g) {
    delete g;
    return IRGL_OK;
}

irgl_status irgl_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    irgl_status st = IRGL_OK;
    for (void *h : g_pinned)
        if (hipHostFree(h) != hipSuccess) st = hip_fail(hipGetLastError());
    g_pinned.clear();
    ++g_pinned_gen;
    return st;
}

irgl_status irgl_graph_default_delta(irgl_graph g, uint32_t *delta) {
    if (!g || !delta) return IRGL_ERR_INVALID_ARGUMENT;
    *delta = default_delta(g);
    return IRGL_OK;
}

irgl_status irgl_workspace_bytes(irgl_graph g, int32_t kind, int32_t with_parent,
                                 const irgl_config *cfg, size_t *bytes) {
    if (!g || !bytes) return IRGL_ERR_INVALID_ARGUMENT;
    if (kind != IRGL_KIND_BFS && kind != IRGL_KIND_SSSP) return IRGL_ERR_INVALID_ARGUMENT;
    Cfg c;
    irgl_status st = resolve(g, kind, cfg, &c);
    if (st) return st;
    *bytes = layout(g, kind, c, with_parent != 0).total;
    return IRGL_OK;
}

irgl_status irgl_bfs(irgl_graph g, int32_t src, uint32_t *level, int32_t *parent, void *ws,
                     size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_config *cfg) {
    return run(IRGL_KIND_BFS, g, src, level, parent, ws, ws_bytes, stream, dstats, cfg);
}

irgl_status irgl_sssp(irgl_graph g, int32_t src, uint32_t *dist, int32_t *parent, void *ws,
                      size_t ws_bytes, void *stream, irgl_stats *dstats, const irgl_config *cfg) {
    return run(IRGL_KIND_SSSP, g, src, dist, parent, ws, ws_bytes, stream, dstats, cfg);
}

irgl_status irgl_sssp_noalloc(irgl_graph g, int32_t src, uint32_t *dist, int32_t *parent, void *stream,
                              irgl_stats *dstats, const irgl_config *cfg) {
    if (!g || !dist) return IRGL_ERR_INVALID_ARGUMENT;
    if (src < 0 || src >= g->n) return IRGL_ERR_INVALID_ARGUMENT;
    if (!g->w) return IRGL_ERR_NO_WEIGHTS;
    Cfg c;
    irgl_status st = resolve(g, IRGL_KIND_SSSP, cfg, &c);
    if (st) return st;
    // the host-loop form reads worklist sizes back through a pinned host
    // word that the library allocates on a thread's first such query
    if (c.mode == IRGL_MODE_HOST_LOOP) return IRGL_ERR_CONFIG;
    if (layout(g, IRGL_KIND_SSSP, c, parent != nullptr).total > kScratchBytes) return IRGL_ERR_TOO_LARGE;
    void *ws = nullptr;
    st = scratch_address(g->device, &ws);
    if (st) return st;
    // run() lays the workspace out exactly as for irgl_sssp; init_kernel
    // resets every part of it the query reads before writing it
    return run(IRGL_KIND_SSSP, g, src, dist, parent, ws, kScratchBytes, stream, dstats, cfg);
}

irgl_status irgl_query_status(const void *ws, void *stream, irgl_stats *out) {
    if (!ws || !out) return IRGL_ERR_INVALID_ARGUMENT;
    IRGL_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    Ctrl c;
    IRGL_HIP(hipMemcpy(&c, ws, sizeof(Ctrl), hipMemcpyDeviceToHost));
    out->status = static_cast<int32_t>(c.error);
    out->iterations = c.iterations;
    out->items = c.items;
    out->edges = c.edges;
    out->max_frontier = c.max_frontier;
    out->grid = c.grid;
    out->block = c.block;
    out->heavy_pulls = c.pulls;
    out->frontier_edges = c.fedges;
    return IRGL_OK;
}


irgl_status irgl_control_block_sizes(int32_t *sizes, int32_t cap, int32_t *count) {
    if (!count || (cap > 0 && !sizes)) return IRGL_ERR_INVALID_ARGUMENT;
    // T_BFS and T_SSSP from the bodies' own constraints: both are
    // ElasticBlock loop bodies whose nested edge scheduler keeps a per-thread
    // gather window and per-wavefront push queues in LDS (Smem<B>, linear in
    // the workgroup size); the batched control kernel holds both, so its sizes
    // are those (among the sizes it is compiled for) that both admit within
    // the device's per-workgroup LDS.
    const long long l64 = static_cast<long long>(sizeof(Smem<64>));
    const long long l1024 = static_cast<long long>(sizeof(Smem<1024>));
    const int32_t per = static_cast<int32_t>((l1024 - l64 + 959) / 960);
    const int32_t base = static_cast<int32_t>(std::max(0ll, l64 - 64ll * per));
    const irgl_block_constraint body = {IRGL_BLOCK_ELASTIC, 1024, base, per};
    int lds = 0, dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipGetLastError();
    if (lds <= 0) lds = 65536;  // no device: gfx950's per-workgroup LDS limit
    const int32_t compiled[] = {256, 512, 1024};  // batch_kernel<B> instantiations
    int32_t k = 0;
    for (int32_t b : compiled) {
        const irgl_block_constraint ks[3] = {body, body, {IRGL_BLOCK_FIXED, b, 0, 0}};
        int32_t chosen = 0;
        if (irgl_control_block(ks, 3, lds, &chosen) == IRGL_OK) {
            if (k < cap) sizes[k] = b;
            ++k;
        }
    }
    *count = k;
    return IRGL_OK;
}

irgl_status irgl_batch_workspace_bytes(const irgl_task *tasks, int32_t ntasks, const irgl_batch_config *cfg,
                                       size_t *bytes) {
    if (!bytes) return IRGL_ERR_INVALID_ARGUMENT;
    irgl_status st = check_tasks(tasks, ntasks);
    if (st) return st;
    BatchCfg c;
    st = resolve_batch(cfg, &c);
    if (st) return st;
    BatchLayout L;
    st = batch_layout(tasks, ntasks, c, tasks[0].g->device, &L);
    if (st) return st;
    *bytes = L.total;
    return IRGL_OK;
}

irgl_status irgl_batch_submit(const irgl_task *tasks, int32_t ntasks, void *ws, size_t ws_bytes,
                              const irgl_batch_config *cfg, void *stream, irgl_batch *out) {
    if (!out || !ws) return IRGL_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    irgl_status st = check_tasks(tasks, ntasks);
    if (st) return st;
    const int dev = tasks[0].g->device;
    for (int32_t i = 1; i < ntasks; ++i)
        if (tasks[i].g->device != dev) return IRGL_ERR_INVALID_ARGUMENT;
    BatchCfg c;
    st = resolve_batch(cfg, &c);
    if (st) return st;
    BatchLayout L;
    st = batch_layout(tasks, ntasks, c, dev, &L);
    if (st) return st;
    if (ws_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    DeviceInfo di;
    st = device_info(dev, &di);
    if (st) return st;
    int cur = -1;
    IRGL_HIP(hipGetDevice(&cur));
    if (cur != dev) IRGL_HIP(hipSetDevice(dev));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);

    irgl_batch_s *b = new (std::nothrow) irgl_batch_s;
    if (!b) return IRGL_ERR_INVALID_ARGUMENT;
    b->ntasks = ntasks;
    b->stream = s;
    b->waited = false;
    b->host_tasks = nullptr;
    b->dev_stats = reinterpret_cast<Stats *>(base + L.stats);
    if (hipHostMalloc(&b->host_tasks, sizeof(TaskDesc) * ntasks, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        if (b->host_tasks) (void)hipHostFree(b->host_tasks);
        delete b;
        return hip_fail(hipGetLastError());
    }
    // largest first (longest-processing-time order); stats keep task order
    std::vector<int32_t> order(ntasks);
    for (int32_t i = 0; i < ntasks; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t bb) {
        return tasks[a].g->m + tasks[a].g->n > tasks[bb].g->m + tasks[bb].g->n;
    });
    TaskDesc *td = static_cast<TaskDesc *>(b->host_tasks);
    for (int32_t k = 0; k < ntasks; ++k) fill_desc(td[k], tasks[order[k]], b->dev_stats + order[k], c.delta);
    BatchParams bp;
    fill_batch_params(bp, L, base, c, di);
    bp.ntasks = ntasks;
    const int grid = L.teams * bp.team;

    st = IRGL_OK;
    if (hipMemcpyAsync(base + L.tasks, b->host_tasks, sizeof(TaskDesc) * ntasks, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        st = hip_fail(hipGetLastError());
    if (!st) {
        hipLaunchKernelGGL(batch_init_kernel, dim3((L.teams + 255) / 256), dim3(256), 0, s, bp.queue_head,
                           bp.scratch, bp.team_bytes, L.teams);
        if (hipGetLastError() != hipSuccess) st = hip_fail(hipGetLastError());
    }
    if (!st) {
        switch (c.block) {
            case 256: st = launch_batch<256>(bp, grid, s); break;
            case 512: st = launch_batch<512>(bp, grid, s); break;
            default: st = launch_batch<1024>(bp, grid, s); break;
        }
    }
    if (!st && hipEventRecord(b->done, s) != hipSuccess) st = hip_fail(hipGetLastError());
    if (cur != dev) (void)hipSetDevice(cur);
    if (st) {
        (void)hipStreamSynchronize(s);
        (void)hipEventDestroy(b->done);
        (void)hipHostFree(b->host_tasks);
        delete b;
        return st;
    }
    *out = b;
    return IRGL_OK;
}

irgl_status irgl_batch_wait(irgl_batch b, irgl_stats *per_task) {
    if (!b) return IRGL_ERR_INVALID_ARGUMENT;
    IRGL_HIP(hipEventSynchronize(b->done));
    b->waited = true;
    if (per_task)
        IRGL_HIP(hipMemcpy(per_task, b->dev_stats, sizeof(Stats) * b->ntasks, hipMemcpyDeviceToHost));
    return IRGL_OK;
}

irgl_status irgl_batch_free(irgl_batch b) {
    if (!b) return IRGL_OK;
    if (!b->waited) (void)hipEventSynchronize(b->done);
    (void)hipEventDestroy(b->done);
    (void)hipHostFree(b->host_tasks);
    delete b;
    return IRGL_OK;
}

// Server workspace: the teams' regions sized for the graphs below the gang
// threshold, then one gang region sized for the graphs at or above it.
struct ServerPlan {
    BatchLayout L;   // teams (and the common words / per-slot statistics)
    BatchLayout G;   // gang region offsets; G.team_bytes = its size (0: no gang graph)
    size_t gang_off;
    size_t total;
    int64_t small_n, small_m, gang_n, gang_m;
    bool weighted;
};

static irgl_status server_plan(const irgl_graph *graphs, int32_t ngraphs, const BatchCfg &c, int32_t ring_cap,
                               ServerPlan *out) {
    if (!graphs || ngraphs <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    ServerPlan P;
    P.small_n = 1;
    P.small_m = 0;
    P.gang_n = 0;
    P.gang_m = 0;
    P.weighted = false;
    for (int32_t i = 0; i < ngraphs; ++i) {
        if (!graphs[i]) return IRGL_ERR_INVALID_ARGUMENT;
        if (graphs[i]->device != graphs[0]->device) return IRGL_ERR_INVALID_ARGUMENT;
        // with gang_queue any task may run as a gang: the gang region fits every graph
        if (c.gang_queue > 0 || graphs[i]->m >= static_cast<int64_t>(c.gang_edges)) {
            P.gang_n = std::max<int64_t>(P.gang_n, graphs[i]->n);
            P.gang_m = std::max<int64_t>(P.gang_m, graphs[i]->m);
        }
        if (graphs[i]->m < static_cast<int64_t>(c.gang_edges)) {
            P.small_n = std::max<int64_t>(P.small_n, graphs[i]->n);
            P.small_m = std::max<int64_t>(P.small_m, graphs[i]->m);
        }
        P.weighted |= graphs[i]->w != nullptr;
    }
    irgl_status st =
        team_layout(P.small_n, P.small_m, P.weighted, true, ring_cap, c, graphs[0]->device, &P.L, true);
    if (st) return st;
    P.G = P.L;
    if (P.gang_n > 0) region_layout(P.gang_n, P.gang_m, P.weighted, c.t_grid, c.block, &P.G);
    else region_layout(1, 0, false, 0, c.block, &P.G);  // the gang control block is always there (exit gangs)
    P.gang_off = P.L.total;
    P.total = P.gang_off + P.G.team_bytes;
    *out = P;
    return IRGL_OK;
}

irgl_status irgl_batch_open_bytes(const irgl_graph *graphs, int32_t ngraphs, const irgl_batch_config *cfg,
                                  int32_t ring_cap, size_t *bytes) {
    if (!bytes || ring_cap <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    BatchCfg c;
    irgl_status st = resolve_batch(cfg, &c);
    if (st) return st;
    ServerPlan P;
    st = server_plan(graphs, ngraphs, c, ring_cap, &P);
    if (st) return st;
    *bytes = P.total;
    return IRGL_OK;
}

irgl_status irgl_batch_open(const irgl_graph *graphs, int32_t ngraphs, const irgl_batch_config *cfg,
                            int32_t ring_cap, uint32_t idle_ms, void *ws, size_t ws_bytes, void *stream,
                            irgl_server *out) {
    if (!out || !ws || ring_cap <= 0) return IRGL_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    BatchCfg c;
    irgl_status st = resolve_batch(cfg, &c);
    if (st) return st;
    ServerPlan P;
    st = server_plan(graphs, ngraphs, c, ring_cap, &P);
    if (st) return st;
    const BatchLayout &L = P.L;
    const int dev = graphs[0]->device;
    if (ws_bytes < P.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    // a team waits at its barrier while its leader polls for work, and team 0
    // ends an idle launch after idle_ms: keep that well inside the watchdog
    if (idle_ms == 0) idle_ms = 50u;
    if (idle_ms > c.watchdog_ms / 4) return IRGL_ERR_CONFIG;
    DeviceInfo di;
    st = device_info(dev, &di);
    if (st) return st;
    irgl_server_s *sv = new (std::nothrow) irgl_server_s;
    ServerParams *sp = new (std::nothrow) ServerParams;
    uint64_t *acked = new (std::nothrow) uint64_t[ring_cap]();
    if (!sv || !sp || !acked) {
        delete sv;
        delete sp;
        delete[] acked;
        return IRGL_ERR_INVALID_ARGUMENT;
    }
    sv->acked = acked;
    const size_t ring_b = align_up(sizeof(TaskDesc) * ring_cap);
    const size_t done_b = align_up(4ull * ring_cap);
    const size_t stats_b = align_up(sizeof(Stats) * ring_cap);
    const size_t host_b = ring_b + 256 + done_b + stats_b;
    void *hm = nullptr;
    if (hipHostMalloc(&hm, host_b, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        delete[] acked;
        delete sv;
        delete sp;
        return hip_fail(hipGetLastError());
    }
    std::memset(hm, 0, host_b);
    char *h = static_cast<char *>(hm);
    char *base = static_cast<char *>(ws);
    fill_batch_params(sp->bp, L, base, c, di);
    sp->bp.ntasks = 0;
    sp->gang = sp->bp;
    sp->gang.scratch = base + P.gang_off;
    sp->gang.team_bytes = P.G.team_bytes;
    sp->gang.off_wl0 = P.G.off_wl0;
    sp->gang.off_wl1 = P.G.off_wl1;
    sp->gang.off_stamp = P.G.off_stamp;
    sp->gang.off_shadow = P.G.off_shadow;
    sp->gang.off_far0 = P.G.off_far0;
    sp->gang.off_far1 = P.G.off_far1;
    sp->gang.off_far_flag = P.G.off_far_flag;
    sp->gang.off_expd = P.G.off_expd;
    sp->gang.off_visited = P.G.off_visited;
    sp->gang.off_hub_v = P.G.off_hub_v;
    sp->gang.off_hub_base = P.G.off_hub_base;
    sp->gang.cap = P.G.cap;
    sp->gang.hub_cap = P.G.hub_cap;
    sp->gang.team = L.teams * L.team;
    sp->ring = reinterpret_cast<TaskDesc *>(h);
    sp->tail = reinterpret_cast<uint32_t *>(h + ring_b);
    sp->stop = reinterpret_cast<uint32_t *>(h + ring_b + 128);
    sp->start_fails = reinterpret_cast<uint32_t *>(h + ring_b + 64);
    sp->done = reinterpret_cast<uint32_t *>(h + ring_b + 256);
    sp->host_stats = reinterpret_cast<Stats *>(h + ring_b + 256 + done_b);
    sp->head = reinterpret_cast<unsigned long long *>(base + L.queue);
    sp->ring_cap = static_cast<uint32_t>(ring_cap);
    sp->idle_ticks = static_cast<unsigned long long>(idle_ms) * di.wallclock_khz;
    sp->start_ticks = static_cast<unsigned long long>(kServerStartMs) * di.wallclock_khz;
    sv->device = dev;
    sv->stream = static_cast<hipStream_t>(stream);
    sv->launched = false;
    sv->block = c.block;
    sv->grid = L.teams * L.team;
    sv->delta = c.delta;
    sv->ring_cap = ring_cap;
    sv->next_ticket = 0;
    sv->dev_head = sp->head;
    sv->dev_stats = reinterpret_cast<Stats *>(base + L.stats);
    sv->sssp_ok = P.weighted;
    sv->small_n = P.small_n;
    sv->small_m = P.small_m;
    sv->gang_n = P.gang_n;
    sv->gang_m = P.gang_m;
    sv->gang_edges = c.gang_edges;
    sv->gang_queue = c.gang_queue;
    sv->completed = 0;
    sv->launches = 0;
    sv->host_mem = hm;
    sv->params = sp;
    if (hipEventCreateWithFlags(&sv->ran, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(hm);
        delete[] acked;
        delete sv;
        delete sp;
        return hip_fail(hipGetLastError());
    }
    // the ring head starts at 0 and is kept across server launches
    hipLaunchKernelGGL(zero_head_kernel, dim3(1), dim3(1), 0, sv->stream, sp->head);
    if (hipGetLastError() != hipSuccess) {
        (void)hipEventDestroy(sv->ran);
        (void)hipHostFree(hm);
        delete[] acked;
        delete sv;
        delete sp;
        return hip_fail(hipGetLastError());
    }
    *out = sv;
    return IRGL_OK;
}

static irgl_status server_launch(irgl_server_s *sv) {
    ServerParams *sp = static_cast<ServerParams *>(sv->params);
    hipLaunchKernelGGL(server_reset_kernel, dim3((sv->grid / sp->bp.team + 1 + 255) / 256), dim3(256), 0,
                       sv->stream, sp->bp.scratch, sp->bp.team_bytes, sv->grid / sp->bp.team,
                       reinterpret_cast<Ctrl *>(sp->gang.scratch), sp->head);
    IRGL_HIP(hipGetLastError());
    irgl_status st;
    switch (sv->block) {
        case 256: st = launch_server<256>(*sp, sv->grid, sv->stream); break;
        case 512: st = launch_server<512>(*sp, sv->grid, sv->stream); break;
        default: st = launch_server<1024>(*sp, sv->grid, sv->stream); break;
    }
    if (st) return st;
    IRGL_HIP(hipEventRecord(sv->ran, sv->stream));
    sv->launched = true;
    ++sv->launches;
    return IRGL_OK;
}

// Launch the server kernel if none is running (it ends after idle_ms).
static irgl_status server_kick(irgl_server_s *sv, bool check_pending) {
    if (sv->launched) {
        const hipError_t q = hipEventQuery(sv->ran);
        if (q == hipErrorNotReady) return IRGL_OK;  // still running: it will see the new tail
        if (q != hipSuccess) return hip_fail(q);
    }
    ServerParams *sp = static_cast<ServerParams *>(sv->params);
    if (check_pending) {
        unsigned long long hw = 0;
        IRGL_HIP(hipMemcpy(&hw, sv->dev_head, 8, hipMemcpyDeviceToHost));
        const uint32_t tail = __atomic_load_n(sp->tail, __ATOMIC_ACQUIRE);
        if (static_cast<uint32_t>(hw) >= tail) return IRGL_OK;
    }
    return server_launch(sv);
}

irgl_status irgl_batch_enqueue(irgl_server s, const irgl_task *task, uint64_t *ticket) {
    if (!s || !task || !ticket) return IRGL_ERR_INVALID_ARGUMENT;
    irgl_status st = check_tasks(task, 1);
    if (st) return st;
    if (task->g->device != s->device) return IRGL_ERR_INVALID_ARGUMENT;
    ServerParams *sp = static_cast<ServerParams *>(s->params);
    const uint64_t inflight = s->next_ticket - s->completed;
    const bool gang = task->g->m >= static_cast<int64_t>(s->gang_edges) ||
                      (s->gang_queue > 0 && inflight < s->gang_queue);
    if (task->kind == IRGL_KIND_SSSP && !s->sssp_ok) return IRGL_ERR_TOO_LARGE;
    if (gang ? (task->g->n > s->gang_n || task->g->m > s->gang_m)
             : (task->g->n > s->small_n || task->g->m > s->small_m))
        return IRGL_ERR_TOO_LARGE;
    const uint64_t t = s->next_ticket;
    const uint32_t slot = static_cast<uint32_t>(t % static_cast<uint64_t>(s->ring_cap));
    // a slot is reused only after its previous task was reported done by irgl_batch_poll
    if (t >= static_cast<uint64_t>(s->ring_cap) && s->acked[slot] != t - static_cast<uint64_t>(s->ring_cap) + 1)
        return IRGL_ERR_BUSY;
    if (t >= 0xFFFFFFF0ull) return IRGL_ERR_BUSY;  // 32-bit ring counters exhausted
    fill_desc(sp->ring[slot], *task, s->dev_stats + slot, s->delta, gang);
    __atomic_store_n(&sp->done[slot], 0u, __ATOMIC_RELAXED);
    __atomic_store_n(const_cast<uint32_t *>(sp->tail), static_cast<uint32_t>(t + 1), __ATOMIC_RELEASE);
    s->next_ticket = t + 1;
    *ticket = t;
    int cur = -1;
    IRGL_HIP(hipGetDevice(&cur));
    if (cur != s->device) IRGL_HIP(hipSetDevice(s->device));
    st = server_kick(s, false);
    if (cur != s->device) (void)hipSetDevice(cur);
    return st;
}

irgl_status irgl_batch_poll(irgl_server s, uint64_t ticket, irgl_stats *st, int32_t *done) {
    if (!s || !done || ticket >= s->next_ticket) return IRGL_ERR_INVALID_ARGUMENT;
    ServerParams *sp = static_cast<ServerParams *>(s->params);
    const uint32_t slot = static_cast<uint32_t>(ticket % static_cast<uint64_t>(s->ring_cap));
    const uint32_t d = __atomic_load_n(&sp->done[slot], __ATOMIC_ACQUIRE);
    if (d == static_cast<uint32_t>(ticket + 1)) {
        if (st) std::memcpy(st, &sp->host_stats[slot], sizeof(irgl_stats));
        if (s->acked[slot] != ticket + 1) ++s->completed;
        s->acked[slot] = ticket + 1;
        *done = 1;
        return IRGL_OK;
    }
    *done = 0;
    if (ticket + static_cast<uint64_t>(s->ring_cap) < s->next_ticket) return IRGL_ERR_INVALID_ARGUMENT;
    int cur = -1;
    IRGL_HIP(hipGetDevice(&cur));
    if (cur != s->device) IRGL_HIP(hipSetDevice(s->device));
    const irgl_status k = server_kick(s, true);
    if (cur != s->device) (void)hipSetDevice(cur);
    return k;
}

irgl_status irgl_batch_launches(irgl_server s, uint64_t *launches, uint64_t *gave_up) {
    if (!s || !launches || !gave_up) return IRGL_ERR_INVALID_ARGUMENT;
    const ServerParams *sp = static_cast<const ServerParams *>(s->params);
    *launches = s->launches;
    *gave_up = __atomic_load_n(sp->start_fails, __ATOMIC_ACQUIRE);
    return IRGL_OK;
}

irgl_status irgl_batch_close(irgl_server s) {
    if (!s) return IRGL_OK;
    ServerParams *sp = static_cast<ServerParams *>(s->params);
    __atomic_store_n(const_cast<uint32_t *>(sp->stop), 1u, __ATOMIC_RELEASE);
    if (s->launched) (void)hipEventSynchronize(s->ran);
    (void)hipEventDestroy(s->ran);
    (void)hipHostFree(s->host_mem);
    delete[] s->acked;
    delete sp;
    delete s;
    return IRGL_OK;
}
}  // extern "C"
