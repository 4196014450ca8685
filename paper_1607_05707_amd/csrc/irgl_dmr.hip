// Delaunay mesh refinement: the refine kernel whose per-item critical
// section is the Exclusive construct (Section 3, Exclusive: three phases
// separated by SyncRunningThreads), driven by the pipe of the DMR main loop
// (Section 4.2, Pipe: identify the bad triangles once, then a looping pipe of
// refine and incremental identification among the triangles refine created,
// then one more identification as a sanity check), all in ONE cooperative
// persistent launch (Section 4.3, iteration outlining).
//
// Domain and quality.  The mesh triangulates the unit square; every live
// triangle is kept Delaunay.  A triangle needs work when it is "bad" (its
// smallest angle is below the bound) or when one of its boundary edges is
// encroached (the opposite vertex sees it at more than 90 degrees).
//
// Refinement of one item (a triangle t from the incoming worklist):
//   * an encroached boundary edge of t is split at its midpoint;
//   * otherwise the circumcentre c of a bad t is located by a walk from t;
//     if the walk leaves the domain through a boundary edge, or c lies in
//     the diametral circle of a boundary edge of its cavity, that edge is
//     split instead; otherwise c is inserted;
//   * the cavity of the new point is the connected set of triangles whose
//     circumcircle contains it; it is re-triangulated by joining the point
//     to every edge of the cavity's boundary (Bowyer-Watson), reusing the
//     cavity's slots and taking one or two new ones.
// The triangles an item must own are its cavity and the triangles just
// outside it (their neighbour entries change).  Exclusive claims them in
// three phases: race (every claimant writes its id), priority check (a
// claimant overwrites any element held by a lower priority, i.e. a larger
// id, with an atomic minimum), check (a claimant that still holds every
// element wins).  The claimant with the smallest id in any conflict wins all
// of its elements, so every round makes progress.  Losers go back to the
// worklist (the Else branch of the construct).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "irgl.h"
#include "irgl_device.h"

namespace irgl_shared {
irgl_status note_hip_failure(hipError_t e);
}  // namespace irgl_shared

namespace irgl {
namespace dmr {

constexpr int kMaxCav = 64;         // cavity triangles of one insertion
constexpr int kMaxOuter = kMaxCav + 2;  // triangles just outside it (one per boundary edge)
constexpr int kMaxWalk = 1 << 16;   // triangles a point location may visit
constexpr int kQ = 256;             // LDS push-queue entries per wavefront

// Counters of one launch (one 128-byte line each for the hot ones).
struct alignas(128) Counters {
    uint32_t out[3];       // rotating out-worklist counters (invocation i pushes out[i % 3])
    uint32_t pad0[29];
    uint32_t npts;         // points in use (atomic: new points)
    uint32_t pad1[31];
    uint32_t ntri;         // triangle slots in use (atomic: new slots)
    uint32_t pad2[31];
    unsigned long long refined;    // items popped by refine
    unsigned long long conflicts;  // items that lost their Exclusive section
    uint32_t inserted;     // circumcentres inserted
    uint32_t splits;       // boundary edges split
    uint32_t max_cavity;
    uint32_t rounds;       // Exclusive rounds (three phases each)
    uint32_t final_bad;    // triangles needing work after the loop (sanity check)
    uint32_t pad3[23];
};

struct Params {
    double2 *pts;
    int4 *tri;
    int4 *nbr;
    uint32_t pcap, tcap;
    uint32_t *lock;
    uint32_t *stamp;
    int32_t *wl[2];
    Ctrl *ctrl;
    Counters *cnt;
    double cos2;            // squared cosine of the angle bound
    uint32_t max_inv;
    unsigned long long wd_ticks;
    uint32_t barrier;
    irgl_dmr_stats *dstats;
};

// ---------------------------------------------------------------------------
// Geometry (double precision; the mesh keeps every triangle counter-clockwise)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double orient(double2 a, double2 b, double2 c) {
    return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// > 0 when d is strictly inside the circle through the counter-clockwise
// triangle (a, b, c)
__device__ __forceinline__ double incircle(double2 a, double2 b, double2 c, double2 d) {
    const double ax = a.x - d.x, ay = a.y - d.y;
    const double bx = b.x - d.x, by = b.y - d.y;
    const double cx = c.x - d.x, cy = c.y - d.y;
    const double al = ax * ax + ay * ay, bl = bx * bx + by * by, cl = cx * cx + cy * cy;
    return ax * (by * cl - bl * cy) - ay * (bx * cl - bl * cx) + al * (bx * cy - by * cx);
}

__device__ __forceinline__ double2 circumcentre(double2 a, double2 b, double2 c) {
    const double bx = b.x - a.x, by = b.y - a.y;
    const double cx = c.x - a.x, cy = c.y - a.y;
    const double d = 2.0 * (bx * cy - by * cx);
    const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
    return make_double2(a.x + (cy * b2 - by * c2) / d, a.y + (bx * c2 - cx * b2) / d);
}

__device__ __forceinline__ double2 midpoint(double2 a, double2 b) {
    return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
}

__device__ __forceinline__ int vtx(const int4 &t, int i) { return i == 0 ? t.x : (i == 1 ? t.y : t.z); }
__device__ __forceinline__ int nbi(const int4 &n, int i) { return i == 0 ? n.x : (i == 1 ? n.y : n.z); }

// Smallest angle below the bound: at some corner the two edge vectors have a
// positive dot product whose square exceeds cos^2(bound) |u|^2 |w|^2.
__device__ __forceinline__ bool is_bad(double2 a, double2 b, double2 c, double cos2) {
    const double2 P[3] = {a, b, c};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 o = P[k], u1 = P[(k + 1) % 3], w1 = P[(k + 2) % 3];
        const double ux = u1.x - o.x, uy = u1.y - o.y, wx = w1.x - o.x, wy = w1.y - o.y;
        const double dot = ux * wx + uy * wy;
        bad |= dot > 0.0 && dot * dot > cos2 * (ux * ux + uy * uy) * (wx * wx + wy * wy);
    }
    return bad;
}

// Boundary edge i of t is encroached when its opposite vertex sees it at
// more than 90 degrees.  Returns that edge, or -1.
__device__ __forceinline__ int encroached_edge(const int4 &n, double2 a, double2 b, double2 c) {
    const double2 P[3] = {a, b, c};
    int e = -1;
#pragma unroll
    for (int i = 2; i >= 0; --i) {
        if (nbi(n, i) >= 0) continue;
        const double2 u = P[i], v = P[(i + 1) % 3], o = P[(i + 2) % 3];
        if ((u.x - o.x) * (v.x - o.x) + (u.y - o.y) * (v.y - o.y) < 0.0) e = i;
    }
    return e;
}

__device__ __forceinline__ bool needs_work(const Params &p, int t) {
    const int4 v = p.tri[t];
    if (!v.w) return false;
    const int4 n = p.nbr[t];
    const double2 a = p.pts[v.x], b = p.pts[v.y], c = p.pts[v.z];
    return encroached_edge(n, a, b, c) >= 0 || is_bad(a, b, c, p.cos2);
}

// ---------------------------------------------------------------------------
// One item of the refine kernel.
// ---------------------------------------------------------------------------
enum : int { kIdle = 0, kClaim = 1 };

struct Item {
    int state;
    uint32_t id;       // priority of the Exclusive section: smaller wins
    int t;             // the popped triangle
    double2 p;         // the point to insert
    int seg_a, seg_b;  // split boundary edge (seg_a -1: inserting a circumcentre)
    int nc, no;        // cavity / outer triangles
    int cav[kMaxCav];
    int outer[kMaxOuter];
};

__device__ __forceinline__ bool in_list(const int *l, int n, int x) {
    for (int k = 0; k < n; ++k)
        if (l[k] == x) return true;
    return false;
}

// Cavity of point q from triangle `start`: breadth-first over neighbours
// whose circumcircle strictly contains q.  False on overflow.
__device__ bool build_cavity(const Params &p, Item &it, int start, double2 q) {
    it.nc = 1;
    it.cav[0] = start;
    for (int k = 0; k < it.nc; ++k) {
        const int4 n = p.nbr[it.cav[k]];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int y = nbi(n, i);
            if (y < 0 || in_list(it.cav, it.nc, y)) continue;
            const int4 ty = p.tri[y];
            if (incircle(p.pts[ty.x], p.pts[ty.y], p.pts[ty.z], q) > 0.0) {
                if (it.nc == kMaxCav) return false;
                it.cav[it.nc++] = y;
            }
        }
    }
    return true;
}

// Decide what the item does and build its cavity.  The mesh is not written
// by anybody during this phase.
__device__ void prepare(const Params &p, Item &it) {
    const int t = it.t;
    const int4 v = p.tri[t];
    if (!v.w) return;
    const int4 n = p.nbr[t];
    const double2 a = p.pts[v.x], b = p.pts[v.y], c = p.pts[v.z];
    int start = t;
    it.seg_a = -1;
    const int e = encroached_edge(n, a, b, c);
    if (e >= 0) {
        it.seg_a = vtx(v, e);
        it.seg_b = vtx(v, (e + 1) % 3);
    } else if (is_bad(a, b, c, p.cos2)) {
        const double2 q = circumcentre(a, b, c);
        // visibility walk towards q; it leaves the domain through a boundary edge
        int cur = t;
        bool found = false;
        for (int step = 0; step < kMaxWalk && !found && it.seg_a < 0; ++step) {
            const int4 tv = p.tri[cur];
            const int4 tn = p.nbr[cur];
            const double2 P[3] = {p.pts[tv.x], p.pts[tv.y], p.pts[tv.z]};
            int go = -1;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (go < 0 && orient(P[i], P[(i + 1) % 3], q) < 0.0) go = i;
            if (go < 0) {
                found = true;
            } else if (nbi(tn, go) < 0) {
                it.seg_a = vtx(tv, go);
                it.seg_b = vtx(tv, (go + 1) % 3);
                start = cur;
            } else {
                cur = nbi(tn, go);
            }
        }
        if (!found && it.seg_a < 0) {
            set_error(p.ctrl, kErrInternal, false);  // the walk did not end
            return;
        }
        if (found) {
            if (!build_cavity(p, it, cur, q)) {
                set_error(p.ctrl, kErrOverflow, false);
                return;
            }
            // a circumcentre inside the diametral circle of a boundary edge of
            // its cavity would encroach it: split that edge instead
            for (int k = 0; k < it.nc && it.seg_a < 0; ++k) {
                const int x = it.cav[k];
                const int4 xv = p.tri[x];
                const int4 xn = p.nbr[x];
                for (int i = 0; i < 3 && it.seg_a < 0; ++i) {
                    if (nbi(xn, i) >= 0) continue;
                    const double2 u = p.pts[vtx(xv, i)], w = p.pts[vtx(xv, (i + 1) % 3)];
                    const double2 m = midpoint(u, w);
                    const double r2 = 0.25 * ((u.x - w.x) * (u.x - w.x) + (u.y - w.y) * (u.y - w.y));
                    if ((q.x - m.x) * (q.x - m.x) + (q.y - m.y) * (q.y - m.y) < r2) {
                        it.seg_a = vtx(xv, i);
                        it.seg_b = vtx(xv, (i + 1) % 3);
                        start = x;
                    }
                }
            }
            if (it.seg_a < 0) it.p = q;
        }
    } else {
        return;  // fixed meanwhile by another insertion
    }
    if (it.seg_a >= 0) {
        it.p = midpoint(p.pts[it.seg_a], p.pts[it.seg_b]);
        if (!build_cavity(p, it, start, it.p)) {
            set_error(p.ctrl, kErrOverflow, false);
            return;
        }
    }
    // the triangles just outside the cavity
    it.no = 0;
    for (int k = 0; k < it.nc; ++k) {
        const int4 xn = p.nbr[it.cav[k]];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int y = nbi(xn, i);
            if (y < 0 || in_list(it.cav, it.nc, y)) continue;
            if (it.no == kMaxOuter) {  // more bordering triangles than a disk-shaped cavity has
                set_error(p.ctrl, kErrInternal, false);
                return;
            }
            it.outer[it.no++] = y;
        }
    }
    it.state = kClaim;
}

// Exclusive, phase 1 (race): write this item's id into every element.
__device__ __forceinline__ void race(const Params &p, const Item &it) {
    for (int k = 0; k < it.nc; ++k) store_agent(&p.lock[it.cav[k]], it.id);
    for (int k = 0; k < it.no; ++k) store_agent(&p.lock[it.outer[k]], it.id);
}

// Phase 2 (priority check): take back every element held by a larger id.
__device__ __forceinline__ void priority_check(const Params &p, const Item &it) {
    for (int k = 0; k < it.nc + it.no; ++k) {
        uint32_t *l = &p.lock[k < it.nc ? it.cav[k] : it.outer[k - it.nc]];
        if (load_agent(l) > it.id) atomicMin(l, it.id);
    }
}

// Phase 3 (check): does this item still hold every element?
__device__ __forceinline__ bool holds_all(const Params &p, const Item &it) {
    bool all = true;
    for (int k = 0; k < it.nc + it.no && all; ++k)
        all = load_agent(&p.lock[k < it.nc ? it.cav[k] : it.outer[k - it.nc]]) == it.id;
    return all;
}

// The winner's critical section: insert it.p and re-triangulate the cavity.
// New triangles (and the popped triangle) are left in `made` for pushing.
__device__ int retriangulate(const Params &p, Item &it, int *made) {
    // edges of the cavity's boundary, counter-clockwise around the cavity
    int ea[kMaxOuter], eb[kMaxOuter], ey[kMaxOuter];
    int k = 0;
    for (int j = 0; j < it.nc; ++j) {
        const int4 xv = p.tri[it.cav[j]];
        const int4 xn = p.nbr[it.cav[j]];
        for (int i = 0; i < 3; ++i) {
            const int y = nbi(xn, i);
            if (y >= 0 && in_list(it.cav, it.nc, y)) continue;
            const int a = vtx(xv, i), b = vtx(xv, (i + 1) % 3);
            if (y < 0 && a == it.seg_a && b == it.seg_b) continue;  // the split edge itself
            if (k == kMaxOuter) {
                set_error(p.ctrl, kErrOverflow, false);
                return 0;
            }
            ea[k] = a;
            eb[k] = b;
            ey[k] = y;
            ++k;
        }
    }
    // a star-shaped cavity gives counter-clockwise new triangles
    for (int j = 0; j < k; ++j) {
        if (!(orient(p.pts[ea[j]], p.pts[eb[j]], it.p) > 0.0)) {
            set_error(p.ctrl, kErrInternal, false);
            return 0;
        }
    }
    if (k <= it.nc) {
        set_error(p.ctrl, kErrInternal, false);
        return 0;
    }
    const uint32_t pid = atomicAdd(&p.cnt->npts, 1u);
    const uint32_t extra = static_cast<uint32_t>(k - it.nc);
    const uint32_t base = atomicAdd(&p.cnt->ntri, extra);
    if (pid >= p.pcap || base + extra > p.tcap || base + extra < base) {
        set_error(p.ctrl, kErrOverflow, true);
        return 0;
    }
    p.pts[pid] = it.p;
    int slot[kMaxOuter];
    for (int j = 0; j < k; ++j) slot[j] = j < it.nc ? it.cav[j] : static_cast<int>(base) + (j - it.nc);
    for (int j = 0; j < k; ++j) {
        int n1 = -1, n2 = -1;  // across (b_j, p) and (p, a_j)
        for (int i = 0; i < k; ++i) {
            if (ea[i] == eb[j]) n1 = slot[i];
            if (eb[i] == ea[j]) n2 = slot[i];
        }
        p.tri[slot[j]] = make_int4(ea[j], eb[j], static_cast<int>(pid), 1);
        p.nbr[slot[j]] = make_int4(ey[j], n1, n2, 0);
        const int y = ey[j];
        if (y >= 0) {
            // the outside triangle's entry for the reversed edge now names the new triangle
            const int4 yv = p.tri[y];
            int4 yn = p.nbr[y];
            if (yv.x == eb[j] && yv.y == ea[j]) yn.x = slot[j];
            else if (yv.y == eb[j] && yv.z == ea[j]) yn.y = slot[j];
            else yn.z = slot[j];
            p.nbr[y] = yn;
        }
        made[j] = slot[j];
    }
    atomicAdd(it.seg_a >= 0 ? &p.cnt->splits : &p.cnt->inserted, 1u);
    atomicMax(&p.cnt->max_cavity, static_cast<uint32_t>(it.nc));
    return k;
}

// ---------------------------------------------------------------------------
// Pushes into the pipe's out worklist, at most once per invocation per
// triangle (push stamp = invocation + 1).  All lanes of a wavefront call it.
// ---------------------------------------------------------------------------
struct Out {
    WaveQueue<kQ> q;
    uint32_t *cnt;
    int32_t *buf;
    uint32_t cap;
    Ctrl *ctrl;
    uint32_t tag;
    __device__ __forceinline__ void push(bool pred, int t, const Params &p) {
        if (pred) pred = atomicExch(&p.stamp[t], tag) != tag;
        q.push(pred, t, cnt, buf, cap, ctrl);
    }
};

struct Smem {
    int q[4][kQ];  // up to 256 threads per workgroup
    int fill[4];
    uint32_t base;
    int flag;
};

template <int B>
__device__ __forceinline__ void drain(Out &o, Smem &sm) {
    block_drain<B, kQ>(o.q, sm.fill, &sm.base, o.cnt, o.buf, o.cap, o.ctrl);
}

// identify_bad_triangles: a ForAll over every triangle slot in use.
template <int B>
__device__ void identify(const Params &p, Team tm, Out &o) {
    const uint32_t ntri = min(load_agent(&p.cnt->ntri), p.tcap);  // the counter may pass tcap on overflow
    for (uint32_t base = tm.id * B; base < ntri; base += tm.size * B) {
        const uint32_t t = base + threadIdx.x;
        const bool w = t < ntri && needs_work(p, static_cast<int>(t));
        o.push(w, static_cast<int>(t), p);
    }
}

// incremental_id_bad_triangles: among the triangles refine created.
template <int B>
__device__ void incremental(const Params &p, const int32_t *in, uint32_t in_n, Team tm, Out &o) {
    for (uint32_t base = tm.id * B; base < in_n; base += tm.size * B) {
        const uint32_t i = base + threadIdx.x;
        int t = 0;
        bool w = false;
        if (i < in_n) {
            t = in[i];
            w = needs_work(p, t);
        }
        o.push(w, t, p);
    }
}

// Priority of item i in one invocation: a bijection of the 32-bit item
// index (xor with a per-invocation salt, then an invertible integer mix:
// xor-shifts and multiplications by odd constants), so ids stay distinct
// while neighbouring items, which tend to sit next to each other in the
// worklist, get unrelated priorities and more of them win per round
// (multipliers from Wellons' published 32-bit integer hash search).
__device__ __forceinline__ uint32_t priority(uint32_t i, uint32_t salt) {
    uint32_t x = i ^ salt;
    x ^= x >> 16;
    x *= 0x21F0AAADu;
    x ^= x >> 15;
    x *= 0x735A2D97u;
    x ^= x >> 15;
    return x;
}

// refine: a ForAll over the worklist whose body holds an Exclusive section;
// the loop runs the same number of rounds in every thread (the section's
// three phases are separated by grid barriers).
template <int B>
__device__ bool refine(const Params &p, const int32_t *in, uint32_t in_n, Team tm, BarrierState &bs, Smem &sm,
                       Out &o, uint32_t salt) {
    const uint32_t nthreads = tm.size * B;
    const uint32_t gtid = tm.id * B + threadIdx.x;
    unsigned long long refined = 0, conflicts = 0;
    Item it;
    int made[kMaxOuter];
    for (uint32_t base = 0; base < in_n; base += nthreads) {
        it.state = kIdle;
        it.nc = it.no = 0;
        const uint32_t i = base + gtid;
        if (i < in_n) {
            it.id = priority(i, salt);
            it.t = in[i];
            ++refined;
            prepare(p, it);
            if (it.state == kClaim) race(p, it);
        }
        if (!grid_barrier(p.ctrl, bs, &sm.flag, nullptr, tm)) return false;
        if (it.state == kClaim) priority_check(p, it);
        if (!grid_barrier(p.ctrl, bs, &sm.flag, nullptr, tm)) return false;
        int nmade = 0;
        if (it.state == kClaim) {
            if (holds_all(p, it)) {
                nmade = retriangulate(p, it, made);
            } else {
                ++conflicts;  // Else: back to the worklist
            }
        }
        // push the new triangles and the popped one (refine's out list feeds
        // the incremental identification); wave-uniform trip count
        int most = nmade;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) most = max(most, __shfl_xor(most, d, kWave));
        for (int j = 0; j < most; ++j) o.push(j < nmade, j < nmade ? made[j] : 0, p);
        o.push(it.state == kClaim, it.t, p);
        if (tm.id == 0 && threadIdx.x == 0) atomicAdd(&p.cnt->rounds, 1u);
        if (!grid_barrier(p.ctrl, bs, &sm.flag, nullptr, tm)) return false;
    }
    if (refined) atomicAdd(&p.cnt->refined, refined);
    if (conflicts) atomicAdd(&p.cnt->conflicts, conflicts);
    return true;
}

// The DMR pipe, outlined:
//   Pipe Once {
//     Invoke identify_bad_triangles;
//     Pipe { Invoke refine; Invoke incremental_id_bad_triangles; }
//     Invoke identify_bad_triangles;   (sanity check: must find none)
//   }
// Invocation i pops `in` (count settled by the previous barrier), pushes
// through out[i % 3], which every workgroup reads right after the barrier
// ending i, and clears out[(i + 1) % 3] for the next invocation (last read
// before the barrier ending i - 1); in and out swap after it.
template <int B>
__global__ __launch_bounds__(B) void dmr_kernel(Params p) {
    __shared__ Smem sm;
    const Team tm = whole_grid();
    BarrierState bs = make_barrier_state(p.wd_ticks, p.barrier);
    const bool lead = tm.id == 0 && threadIdx.x == 0;
    const int wid = threadIdx.x / kWave;
    uint32_t inv = 0, in_n = 0;
    int in_b = 0;
    bool ok = true;
    // 0: first identification, 1: refine, 2: incremental, 3: final check
    int stage = 0;
    while (ok) {
        if (inv >= p.max_inv) {
            if (lead) set_error(p.ctrl, kErrIterLimit, true);
            break;
        }
        if (lead) store_agent(&p.cnt->out[(inv + 1) % 3], 0u);
        Out o{{sm.q[wid], 0}, &p.cnt->out[inv % 3], p.wl[in_b ^ 1], p.tcap, p.ctrl, inv + 1};
        const int32_t *in = p.wl[in_b];
        if (stage == 0 || stage == 3) identify<B>(p, tm, o);
        else if (stage == 1) ok = refine<B>(p, in, in_n, tm, bs, sm, o, inv * 0x9E3779B9u);
        else incremental<B>(p, in, in_n, tm, o);
        if (!ok) break;
        drain<B>(o, sm);
        if (!grid_barrier(p.ctrl, bs, &sm.flag, nullptr, tm)) break;
        const uint32_t produced = min(load_agent(&p.cnt->out[inv % 3]), p.tcap);
        ++inv;
        if (stage == 3) {
            if (lead) p.cnt->final_bad = produced;
            break;
        }
        in_b ^= 1;
        in_n = produced;
        if (stage == 0 || stage == 2) stage = in_n > 0 ? 1 : 3;  // the looping pipe runs while its worklist has items
        else stage = 2;
    }
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(&p.ctrl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == tm.size - 1 && p.dstats) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            irgl_dmr_stats *st = p.dstats;
            st->status = static_cast<int32_t>(load_agent(&p.ctrl->error));
            st->invocations = inv;
            st->rounds = p.cnt->rounds;
            st->block = B;
            st->grid = static_cast<int32_t>(tm.size);
            st->refined = p.cnt->refined;
            st->conflicts = p.cnt->conflicts;
            st->inserted = p.cnt->inserted;
            st->splits = p.cnt->splits;
            st->npts = static_cast<int32_t>(min(load_agent(&p.cnt->npts), p.pcap));
            st->ntri = static_cast<int32_t>(min(load_agent(&p.cnt->ntri), p.tcap));
            st->final_bad = p.cnt->final_bad;
            st->max_cavity = p.cnt->max_cavity;
        }
    }
}

// Fresh launch: control block, counters, push stamps.
__global__ void dmr_init_kernel(Ctrl *c, Counters *k, uint32_t *stamp, uint32_t tcap, uint32_t npts, uint32_t ntri) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t t = g; t < tcap; t += gridDim.x * blockDim.x) stamp[t] = 0u;
    if (g == 0) {
        reset_barrier_words(c);
        c->error = 0;
        c->fatal = 0;
        c->done = 0;
        for (int i = 0; i < 3; ++i) k->out[i] = 0;
        k->npts = npts;
        k->ntri = ntri;
        k->refined = 0;
        k->conflicts = 0;
        k->inserted = 0;
        k->splits = 0;
        k->max_cavity = 0;
        k->rounds = 0;
        k->final_bad = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kA = 256;
constexpr size_t up(size_t x) { return (x + kA - 1) / kA * kA; }

struct Layout {
    size_t ctrl, cnt, wl0, wl1, lock, stamp, total;
};

Layout layout(uint32_t tcap) {
    Layout L;
    const size_t tb = up(static_cast<size_t>(tcap) * 4);
    L.ctrl = 0;
    L.cnt = up(sizeof(Ctrl));
    L.wl0 = L.cnt + up(sizeof(Counters));
    L.wl1 = L.wl0 + tb;
    L.lock = L.wl1 + tb;
    L.stamp = L.lock + tb;
    L.total = L.stamp + tb;
    return L;
}

#define DMR_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return irgl_shared::note_hip_failure(e_); \
    } while (0)

irgl_status check_mesh_args(const irgl_mesh *m) {
    if (!m || !m->pts || !m->tri || !m->nbr) return IRGL_ERR_INVALID_ARGUMENT;
    if (m->npts < 3 || m->ntri < 1 || m->pcap < m->npts || m->tcap < m->ntri) return IRGL_ERR_INVALID_ARGUMENT;
    if (m->tcap >= (1 << 30) || m->pcap >= (1 << 30)) return IRGL_ERR_INVALID_ARGUMENT;
    return IRGL_OK;
}

template <int B>
irgl_status launch(Params &p, int requested, hipStream_t s, int *grid_out) {
    int dev = 0, cus = 0, per_cu = 0;
    DMR_HIP(hipGetDevice(&dev));
    DMR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    DMR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dmr_kernel<B>, B, 0));
    // at most 6 waves per SIMD are co-resident on gfx950 (the library's cap
    // for every cooperative launch)
    per_cu = std::min(per_cu, std::max(1, 24 / (B / kWave)));
    const int limit = per_cu * cus;
    if (limit <= 0 || requested < 0 || requested > limit) return IRGL_ERR_CONFIG;
    const int grid = requested ? requested : limit;
    void *args[] = {&p};
    DMR_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(dmr_kernel<B>), dim3(grid), dim3(B), args, 0,
                                       s));
    *grid_out = grid;
    return IRGL_OK;
}

}  // namespace dmr
}  // namespace irgl

using namespace irgl::dmr;

extern "C" {

irgl_status irgl_dmr_workspace_bytes(const irgl_mesh *m, size_t *bytes) {
    if (!bytes) return IRGL_ERR_INVALID_ARGUMENT;
    irgl_status st = check_mesh_args(m);
    if (st) return st;
    *bytes = layout(static_cast<uint32_t>(m->tcap)).total;
    return IRGL_OK;
}

irgl_status irgl_dmr_refine(const irgl_mesh *m, void *ws, size_t ws_bytes, const irgl_dmr_config *cfg, void *stream,
                            irgl_dmr_stats *dstats) {
    irgl_status st = check_mesh_args(m);
    if (st) return st;
    if (!ws) return IRGL_ERR_INVALID_ARGUMENT;
    const Layout L = layout(static_cast<uint32_t>(m->tcap));
    if (ws_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
    const double angle = (cfg && cfg->min_angle != 0.0) ? cfg->min_angle : 30.0;
    // no triangle has all its angles above 60 degrees
    if (!(angle > 0.0 && angle < 60.0)) return IRGL_ERR_CONFIG;
    const int block = (cfg && cfg->block) ? cfg->block : 256;
    if (block != 64 && block != 128 && block != 256) return IRGL_ERR_CONFIG;
    if (cfg && (cfg->barrier > IRGL_BARRIER_WORKGROUP || cfg->grid < 0)) return IRGL_ERR_CONFIG;
    const double r = angle * 3.14159265358979323846 / 180.0;
    const double cs = __builtin_cos(r);
    char *b = static_cast<char *>(ws);
    Params p;
    std::memset(&p, 0, sizeof(p));
    p.pts = reinterpret_cast<double2 *>(m->pts);
    p.tri = reinterpret_cast<int4 *>(m->tri);
    p.nbr = reinterpret_cast<int4 *>(m->nbr);
    p.pcap = static_cast<uint32_t>(m->pcap);
    p.tcap = static_cast<uint32_t>(m->tcap);
    p.ctrl = reinterpret_cast<irgl::Ctrl *>(b + L.ctrl);
    p.cnt = reinterpret_cast<Counters *>(b + L.cnt);
    p.wl[0] = reinterpret_cast<int32_t *>(b + L.wl0);
    p.wl[1] = reinterpret_cast<int32_t *>(b + L.wl1);
    p.lock = reinterpret_cast<uint32_t *>(b + L.lock);
    p.stamp = reinterpret_cast<uint32_t *>(b + L.stamp);
    p.cos2 = cs * cs;
    p.max_inv = (cfg && cfg->max_invocations) ? cfg->max_invocations : 100000u;
    int dev = 0, khz = 0;
    DMR_HIP(hipGetDevice(&dev));
    DMR_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const uint32_t wd_ms = (cfg && cfg->watchdog_ms) ? cfg->watchdog_ms : 20000u;
    p.wd_ticks = wd_ms == IRGL_WATCHDOG_IMMEDIATE ? 0ull
                                                  : static_cast<unsigned long long>(wd_ms) * (khz > 0 ? khz : 100000);
    p.barrier = cfg ? cfg->barrier : IRGL_BARRIER_XCD;
    p.dstats = dstats;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int igrid = static_cast<int>(std::min<uint32_t>(4096u, (p.tcap + 255u) / 256u));
    hipLaunchKernelGGL(dmr_init_kernel, dim3(std::max(1, igrid)), dim3(256), 0, s, p.ctrl, p.cnt, p.stamp, p.tcap,
                       static_cast<uint32_t>(m->npts), static_cast<uint32_t>(m->ntri));
    DMR_HIP(hipGetLastError());
    const int requested = cfg ? cfg->grid : 0;
    int grid = 0;
    switch (block) {
        case 64: return launch<64>(p, requested, s, &grid);
        case 128: return launch<128>(p, requested, s, &grid);
        default: return launch<256>(p, requested, s, &grid);
    }
}

}  // extern "C"
