// Per-query parameters and the relax operators (BFS check-and-label, SSSP
// near/far relaxation, SSSP parent pass) of the data-driven hot path.
#pragma once

#include "irgl_device.h"

namespace irgl {


constexpr int kQueueCap = 256;  // LDS staging entries per wavefront
constexpr int kHeavyQ = 64;     // LDS staging entries per wavefront for the SSSP heavy list
constexpr int kUMax = 4;        // largest edges-per-lane-per-round of any operator

// Shared-memory layout of the frontier kernels for workgroup size B.
template <int B>
struct Smem {
    static constexpr int NW = B / kWave;
    int gstart[B];                 // gather tier: first slot of each thread's range (exclusive scan)
    int gr0[B];                    // gather tier: first edge of each thread's range
    int vtx[B];                    // popped vertex of each thread
    uint32_t vval[B];              // its per-vertex value (SSSP distance at pop)
    int wsum[NW];                  // per-wavefront degree sums for the workgroup scan
    int fill[NW];                  // per-wavefront queue fill at the workgroup drain
    int queue[NW][kQueueCap];      // worklist (near) staging
    int queue_far[NW][kQueueCap];  // SSSP far-list staging
    int queue_heavy[NW][kHeavyQ];  // SSSP heavy-list staging (vertices expanded in the current bucket)
    int owner;                     // workgroup-tier vertex owner
    int big_r0, big_r1, big_v;
    uint32_t big_val;
    uint32_t base;
    int flag;
    int hub_h;                     // grid tier: first deferred vertex of this workgroup
    uint32_t tile;                 // next worklist tile of this workgroup
};

struct Params {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    uint32_t *val;        // level (BFS) or dist (SSSP)
    int32_t *parent;      // optional
    uint32_t *stamp;      // SSSP push stamps
    uint32_t *shadow;     // SSSP probe-only copy of dist (never touched by atomics)
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
    int32_t src_orig;     // the source's caller id (parents are caller ids)
    const int32_t *perm;  // relabelled graph: internal id -> caller id, else null
    uint32_t it;          // host-loop mode: the invocation to run
    unsigned long long wd_ticks;
    uint32_t barrier;  // grid-barrier coherence scheme (kBar*)
    const volatile int32_t *abort_flag;
    uint32_t *visited;    // BFS visited / SSSP settled bitmap, ceil(n / 32) words
    uint32_t t_bitmap;    // refresh it once this many new items were popped since the last refresh
    uint32_t trace_len;
    unsigned long long *trace;
    int32_t *far0;        // SSSP far lists (two buffers), n entries each
    int32_t *far1;
    uint32_t *far_flag;   // SSSP: 1 while a vertex is on the far list
    uint32_t far_cap;
    uint32_t delta;       // SSSP threshold step (INF: plain Bellman-Ford)
    uint32_t thresh;      // host-loop mode: current threshold
    uint32_t far_tr;      // host-loop mode: threshold raises so far
    uint32_t refresh;     // host-loop mode: refresh the bitmap in this invocation
    uint32_t *frontier;   // BFS bottom-up: bitmap of the current frontier, or null (top-down only)
    uint32_t *frontier2;  // ... and of the next one (a bottom-up invocation writes it)
    uint32_t do_alpha;    // BFS direction choice (see irgl_config)
    uint32_t do_beta;
    long long m;          // edges of the graph
    uint32_t reduce_all;  // topology-driven loop: 1 = Iterate Until All(unchanged), 0 = While Any(changed)
    // SSSP light/heavy split (rows partitioned at upload: edges lighter than
    // `delta` first): split[v] = first heavy edge of v, or null (no split)
    const int32_t *split;
    uint32_t *expd;       // SSSP: distance of each vertex's last expansion (INF: never), or null
    int32_t *hlist;       // SSSP split: vertices expanded in the current bucket
    uint32_t *hstamp;     // ... and the bucket in which each was last listed
    uint32_t hcap;
    // relabelled graph, outlined loop: map the results to caller ids at the
    // end of the launch (out_caller[o] = val[inv[o]]), or null
    const int32_t *inv;
    uint32_t *out_caller;
    int32_t *parent_caller;
    // SSSP on a split scale-free graph: a threshold raise that finds fewer
    // than (items popped so far) / tail_div vertices on the far list ends the
    // bucketing (threshold = INF: the rest runs in plain Bellman-Ford order);
    // 0 = never
    uint32_t tail_div;
    // SSSP: the shadow distances are 16-bit (saturating at 0xFFFF = "no
    // bound"), half the probe footprint; for graphs whose distances are
    // small (the split scale-free path)
    uint32_t shadow16;
    // SSSP on a split symmetric graph: a bucket whose listed vertices hold at
    // least n / pull_heavy_div heavy edges runs its heavy pass as a pull
    // (every unsettled vertex looks through its own heavy range for the
    // bucket's vertices); 0 = always push
    uint32_t pull_heavy_div;
    // ... and whose listed heavy edges are at least 1 / pull_open_div of the
    // heavy edges of the vertices not listed before (the pull scans those);
    // 0 = no such bound.  heavy_m = heavy edges of the partition.
    uint32_t pull_open_div;
    unsigned long long heavy_m;
    // SSSP with the pull bookkeeping: once 7/8 of the heavy entries have been
    // listed, thresholds rise by step_grow steps at a time; 0 = one step
    uint32_t step_grow;
};

// ---------------------------------------------------------------------------
// Relax operators.  relax(e, d, sv, sval, act) receives U scanned edges
// e[k] = (sv[k] -> d[k]) of this lane, act[k] marking the live ones, and
// leaves act[k] true for each destination that must be pushed.  `tries` /
// `wins` count this lane's claim atomics and the successful ones.
// ---------------------------------------------------------------------------
struct BfsOp {
    static constexpr bool kPush = true;
    static constexpr bool kFar = false;
    // edges per lane per round (memory-level parallelism) and the fewest
    // waves per SIMD the persistent kernel must fit (1: no register cap)
    static constexpr int kU = 4;
    static constexpr int kMinWaves = 1;
    uint32_t *level;
    int32_t *parent;
    const uint32_t *visited;  // bitmap: a set bit means "visited" (never a false positive)
    uint32_t next;            // label of vertices found in this invocation
    const int32_t *perm;      // relabelled graph: parents are stored as caller ids
    __device__ __forceinline__ uint32_t vertex_value(int) const { return 0u; }
    __device__ __forceinline__ bool active(uint32_t) const { return true; }
    __device__ __forceinline__ void relax(const int (&)[kU], const int (&d)[kU], const int (&sv)[kU],
                                          const uint32_t (&)[kU], bool (&act)[kU], bool (&)[kU],
                                          uint32_t &, uint32_t &tries, uint32_t &wins) const {
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
            tries += act[k] ? 1u : 0u;
            if (act[k]) act[k] = atomicCAS(&level[d[k]], kInf, next) == kInf;
            wins += act[k] ? 1u : 0u;
        }
        if (parent) {
#pragma unroll
            for (int k = 0; k < kU; ++k)
                if (act[k]) parent[d[k]] = perm ? perm[sv[k]] : sv[k];
        }
    }
};

// The register cap of a persistent kernel of B threads per workgroup: the
// fewest waves per SIMD that hold as many whole workgroups per compute unit
// (four SIMDs) as a cap of W waves per SIMD would.  Where W waves do not
// divide into whole workgroups (two workgroups of 512 threads fill 4 of 5),
// the looser cap gives the compiler more registers, hence fewer spills, for
// the same co-resident grid.
template <int B, int W>
constexpr int fit_waves() {
    constexpr int per_block = B / kWave;
    constexpr int blocks = (4 * W) / per_block;
    return blocks <= 0 ? W : (blocks * per_block + 3) / 4;
}
static_assert(fit_waves<256, 5>() == 5 && fit_waves<512, 5>() == 4 && fit_waves<1024, 5>() == 4 &&
                  fit_waves<512, 1>() == 1,
              "register cap per workgroup size");

// SSSP relaxation with a near/far split of the worklist (a bucketed,
// delta-stepping order of the same data-driven loop): an improved vertex
// whose new distance is below the current threshold goes to the next
// invocation's worklist ("near", at most once per invocation by the push
// stamp); otherwise to the far list (at most once while it is listed, by
// far_flag).  thresh = INF gives plain bulk-synchronous Bellman-Ford.
struct SsspOp {
    static constexpr bool kPush = true;
    static constexpr bool kFar = true;
    // Measured on RMAT-22: 2 edges per lane and a register cap that fits 5
    // waves per SIMD (1280 workgroups instead of 768) beat 4 edges per lane:
    // each relaxation is a chain of dependent loads, so more waves in flight
    // hide more latency than more edges per wave.
    static constexpr int kU = 2;
    static constexpr int kMinWaves = 5;
    uint32_t *dist;
    const uint32_t *w;
    uint32_t *stamp;
    uint32_t *far_flag;
    uint32_t thresh;
    uint32_t it;
    Ctrl *ctrl;
    const uint32_t *settled;  // bitmap of vertices whose distance is final, or null
    // Probe-only copy of dist: an upper bound of it (every value it ever held
    // was a tentative distance, and distances only fall), written with plain
    // stores after a successful atomicMin and never touched by an atomic, so
    // its lines stay cacheable in L2 while dist's lines, hammered by atomics,
    // do not.  A relaxation that cannot beat the bound cannot improve dist.
    uint32_t *shadow;
    // 1: shadow holds 16-bit values, min(bound, 0xFFFF); 0xFFFF reads as no
    // bound, so a saturated entry only weakens the filter
    uint32_t shadow16 = 0;
    // Light/heavy split (null: every edge is relaxed when its source is
    // expanded).  Rows are partitioned so that edges lighter than the step
    // come first; an expansion relaxes only [row_ptr[v], split[v]) and lists
    // v for the bucket's heavy pass, which relaxes [split[v], row_ptr[v+1])
    // once, with v's final distance, after the bucket has drained.
    const int32_t *split = nullptr;
    // distance of each vertex's last expansion: a popped vertex whose
    // distance equals it has already relaxed its edges with that distance
    uint32_t *expd = nullptr;
    uint32_t *hstamp = nullptr;  // bucket of each vertex's last heavy-list entry
    uint32_t bucket = 0;         // current bucket (threshold raises so far)
    uint32_t heavy = 0;          // 1: this invocation relaxes heavy ranges
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return dist[v]; }
    __device__ __forceinline__ bool active(uint32_t) const { return true; }
    __device__ __forceinline__ void relax(const int (&e)[kU], const int (&d)[kU], const int (&)[kU],
                                          const uint32_t (&dv)[kU], bool (&act)[kU],
                                          bool (&far)[kU], uint32_t &fmin, uint32_t &tries, uint32_t &wins) const {
        uint32_t nd[kU], cur[kU];
        // a settled destination cannot improve (weights >= 1): skip it with an
        // L2-resident bit test instead of a probe of dist[]
        if (settled) {
#pragma unroll
            for (int k = 0; k < kU; ++k) cur[k] = act[k] ? settled[static_cast<uint32_t>(d[k]) >> 5] : 0u;
#pragma unroll
            for (int k = 0; k < kU; ++k) act[k] = act[k] && !(cur[k] & (1u << (d[k] & 31)));
        }
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
        for (int k = 0; k < kU; ++k) {
            if (shadow16) {  // uniform
                const uint32_t h = act[k] ? reinterpret_cast<const uint16_t *>(shadow)[d[k]] : 0u;
                cur[k] = h == 0xFFFFu ? kInf : h;
            } else {
                cur[k] = act[k] ? shadow[d[k]] : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            act[k] = act[k] && nd[k] < cur[k];
            tries += act[k] ? 1u : 0u;
            if (act[k]) act[k] = nd[k] < atomicMin(&dist[d[k]], nd[k]);
            wins += act[k] ? 1u : 0u;
            if (act[k]) {
                if (shadow16) reinterpret_cast<uint16_t *>(shadow)[d[k]] = static_cast<uint16_t>(min(nd[k], 0xFFFFu));
                else shadow[d[k]] = nd[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            far[k] = act[k] && nd[k] >= thresh;
            act[k] = act[k] && nd[k] < thresh;
            if (far[k]) fmin = min(fmin, nd[k]);  // lower bound of the far list
        }
        // near: push d at most once per invocation; far: at most once while listed
#pragma unroll
        for (int k = 0; k < kU; ++k) cur[k] = act[k] ? stamp[d[k]] : (far[k] ? far_flag[d[k]] : it);
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            act[k] = act[k] && cur[k] != it;
            if (act[k]) act[k] = atomicExch(&stamp[d[k]], it) != it;
            far[k] = far[k] && cur[k] == 0u;
            if (far[k]) far[k] = atomicExch(&far_flag[d[k]], 1u) == 0u;
        }
    }
};

// Deterministic SSSP parents after convergence: the smallest-id tight
// predecessor of every reached vertex (unsigned min over -1 = 0xFFFFFFFF).
struct SsspParentOp {
    static constexpr bool kPush = false;
    static constexpr bool kFar = false;
    static constexpr int kU = 4;
    static constexpr int kMinWaves = 1;
    const uint32_t *dist;
    const uint32_t *w;
    int32_t *parent;
    int32_t src;
    const int32_t *perm;  // relabelled graph: the smallest CALLER id wins, stored as a caller id
    __device__ __forceinline__ uint32_t vertex_value(int v) const { return dist[v]; }
    __device__ __forceinline__ bool active(uint32_t dv) const { return dv != kInf; }
    __device__ __forceinline__ void relax(const int (&e)[kU], const int (&d)[kU], const int (&sv)[kU],
                                          const uint32_t (&dv)[kU], bool (&act)[kU], bool (&)[kU],
                                          uint32_t &, uint32_t &, uint32_t &) const {
        uint32_t s[kU], cur[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) s[k] = act[k] ? dv[k] + w[e[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) cur[k] = act[k] ? dist[d[k]] : 0u;
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            if (act[k] && d[k] != src && s[k] == cur[k] && s[k] >= dv[k])
                atomicMin(reinterpret_cast<uint32_t *>(&parent[d[k]]),
                          static_cast<uint32_t>(perm ? perm[sv[k]] : sv[k]));
            act[k] = false;
        }
    }
};

}  // namespace irgl
