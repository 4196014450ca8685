// Host runtime and C ABI of the MI355X BFS/SSSP library (declared in
// include/irgl.h).  It owns no device memory: graphs are borrowed caller
// arrays, per-query state lives in a caller workspace.  It picks block sizes
// and tier thresholds, sizes the co-resident grid with the occupancy API
// (Section 3.4: a grid barrier is safe only when every workgroup is
// resident), and launches either the outlined persistent loop (one
// cooperative launch per query) or the un-outlined host loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>

#include "irgl.h"
#include "irgl_kernels.h"

using namespace irgl;

static_assert(sizeof(Stats) == sizeof(irgl_stats), "irgl_stats layout");
static_assert(offsetof(Stats, edges) == offsetof(irgl_stats, edges), "irgl_stats layout");
static_assert(offsetof(Stats, block) == offsetof(irgl_stats, block), "irgl_stats layout");

struct irgl_graph_s {
    int32_t n;
    int64_t m;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    uint32_t flags;
    int device;
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

constexpr size_t kAlign = 256;
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
};

irgl_status resolve(const irgl_graph_s *g, const irgl_config *c, Cfg *out) {
    Cfg r;
    r.block = (c && c->block) ? c->block : 512;
    if (r.block != 256 && r.block != 512 && r.block != 1024) return IRGL_ERR_CONFIG;
    r.t_wave = (c && c->t_wave) ? c->t_wave : 64;
    r.t_block = (c && c->t_block) ? c->t_block : r.block;
    if (r.t_wave < 1 || r.t_block < r.t_wave) return IRGL_ERR_CONFIG;
    // grid tier: vertices with at least this many edges are split over all
    // workgroups (IRGL_GRID_TIER_OFF disables it)
    r.t_grid = (c && c->t_grid) ? c->t_grid : 8 * r.block * kU;
    if (c && c->t_grid == IRGL_GRID_TIER_OFF) r.t_grid = 0;
    if (r.t_grid < 0 || (r.t_grid > 0 && r.t_grid < r.t_block)) return IRGL_ERR_CONFIG;
    r.grid = c ? c->grid : 0;
    if (r.grid < 0) return IRGL_ERR_CONFIG;
    r.mode = c ? c->mode : IRGL_MODE_PERSISTENT;
    if (r.mode != IRGL_MODE_PERSISTENT && r.mode != IRGL_MODE_HOST_LOOP) return IRGL_ERR_CONFIG;
    const uint32_t n = static_cast<uint32_t>(g->n);
    r.max_iter = (c && c->max_iter) ? c->max_iter : n + 1u;
    r.cap = (c && c->wl_capacity) ? std::min(c->wl_capacity, n) : n;
    r.watchdog_ms = (c && c->watchdog_ms) ? c->watchdog_ms : 20000u;
    r.abort_flag = c ? c->abort_flag : nullptr;
    r.t_bitmap = (c && c->t_bitmap) ? c->t_bitmap : std::max(1u, n / 64u);
    r.trace_len = (c && c->trace) ? c->trace_len : 0u;
    r.trace = (c && c->trace) ? reinterpret_cast<unsigned long long *>(c->trace) : nullptr;
    *out = r;
    return IRGL_OK;
}

struct Layout {
    size_t ctrl, wl0, wl1, stamp, visited, hub_v, hub_base, total;
    uint32_t hub_cap;
};

Layout layout(const irgl_graph_s *g, int kind, const Cfg &c) {
    Layout L;
    L.ctrl = 0;
    L.wl0 = align_up(sizeof(Ctrl));
    L.wl1 = L.wl0 + align_up(static_cast<size_t>(c.cap) * 4);
    L.stamp = L.wl1 + align_up(static_cast<size_t>(c.cap) * 4);
    L.visited = L.stamp + (kind == IRGL_KIND_SSSP ? align_up(static_cast<size_t>(g->n) * 4) : 0);
    const bool bitmap = kind == IRGL_KIND_BFS && c.t_bitmap != IRGL_BITMAP_NEVER;
    L.hub_v = L.visited + (bitmap ? align_up((static_cast<size_t>(g->n) + 31) / 32 * 4) : 0);
    // at most m / t_grid vertices have t_grid or more edges
    L.hub_cap = c.t_grid > 0
                    ? static_cast<uint32_t>(std::min<int64_t>(g->n, g->m / c.t_grid + 1))
                    : 0u;
    L.hub_base = L.hub_v + align_up(static_cast<size_t>(L.hub_cap) * 4);
    L.total = L.hub_base + align_up(static_cast<size_t>(L.hub_cap) * 4);
    return L;
}

template <class K>
irgl_status coresident_grid(K kernel, int block, int dev, int requested, int *grid) {
    DeviceInfo di;
    irgl_status st = device_info(dev, &di);
    if (st) return st;
    int per_cu = 0;
    IRGL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
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

thread_local uint32_t *t_pinned = nullptr;

irgl_status pinned_word(uint32_t **p) {
    if (!t_pinned) {
        void *h = nullptr;
        IRGL_HIP(hipHostMalloc(&h, 64, hipHostMallocDefault));
        t_pinned = static_cast<uint32_t *>(h);
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
        for (;; ++it) {
            if (it >= c.max_iter) {
                hit_limit = 1;
                break;
            }
            p.it = it;
            hipLaunchKernelGGL((level_kernel<B, Op>), dim3(grid), dim3(B), 0, s, p);
            IRGL_HIP(hipGetLastError());
            if (p.t_grid > 0) {
                hipLaunchKernelGGL((hub_level_kernel<B, Op>), dim3(grid), dim3(B), 0, s, p);
                IRGL_HIP(hipGetLastError());
            }
            IRGL_HIP(hipMemcpyAsync(host, &p.ctrl->cnt[(it + 1) % 3], 4, hipMemcpyDeviceToHost, s));
            IRGL_HIP(hipStreamSynchronize(s));
            if (*host == 0) break;
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
    irgl_status st = resolve(g, cfg, &c);
    if (st) return st;
    const Layout L = layout(g, kind, c);
    if (ws_bytes < L.total) return IRGL_ERR_WORKSPACE_TOO_SMALL;
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
    p.val = out;
    p.parent = parent;
    p.ctrl = reinterpret_cast<Ctrl *>(base + L.ctrl);
    p.wl0 = reinterpret_cast<int32_t *>(base + L.wl0);
    p.wl1 = reinterpret_cast<int32_t *>(base + L.wl1);
    p.stamp = kind == IRGL_KIND_SSSP ? reinterpret_cast<uint32_t *>(base + L.stamp) : nullptr;
    p.visited = (kind == IRGL_KIND_BFS && c.t_bitmap != IRGL_BITMAP_NEVER)
                    ? reinterpret_cast<uint32_t *>(base + L.visited) : nullptr;
    p.t_bitmap = c.t_bitmap;
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
    p.src = src;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kind == IRGL_KIND_BFS) st = dispatch_block<BfsOp>(g, p, c, s, kind);
    else st = dispatch_block<SsspOp>(g, p, c, s, kind);
    if (cur != g->device) (void)hipSetDevice(cur);
    return st;
}

__device__ uint32_t g_invalid_flag;

__global__ void clear_flag_kernel() { g_invalid_flag = 0u; }

}  // namespace

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

irgl_status irgl_graph_upload(const irgl_csr *csr, irgl_graph *out) {
    if (!csr || !out) return IRGL_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (csr->n <= 0 || csr->m < 0 || csr->m >= (int64_t(1) << 31)) return IRGL_ERR_INVALID_ARGUMENT;
    if (!csr->row_ptr || (csr->m > 0 && !csr->col)) return IRGL_ERR_INVALID_ARGUMENT;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return IRGL_ERR_NO_DEVICE;
    }
    int dev = 0;
    IRGL_HIP(hipGetDevice(&dev));
    if (csr->flags & IRGL_VALIDATE) {
        hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, 0);
        IRGL_HIP(hipGetLastError());
        uint32_t *flag = nullptr;
        IRGL_HIP(hipGetSymbolAddress(reinterpret_cast<void **>(&flag), HIP_SYMBOL(g_invalid_flag)));
        const int grid = std::min<int64_t>(4096, std::max<int64_t>(1, (csr->m + 255) / 256));
        hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(256), 0, 0, csr->n, csr->m, csr->row_ptr,
                           csr->col, csr->w, flag);
        IRGL_HIP(hipGetLastError());
        uint32_t bad = 0;
        IRGL_HIP(hipMemcpy(&bad, flag, 4, hipMemcpyDeviceToHost));
        if (bad) return IRGL_ERR_INVALID_GRAPH;
    }
    irgl_graph_s *g = new (std::nothrow) irgl_graph_s;
    if (!g) return IRGL_ERR_INVALID_ARGUMENT;
    g->n = csr->n;
    g->m = csr->m;
    g->row_ptr = csr->row_ptr;
    g->col = csr->col;
    g->w = csr->w;
    g->flags = csr->flags;
    g->device = dev;
    *out = g;
    return IRGL_OK;
}

irgl_status irgl_graph_free(irgl_graph g) {
    delete g;
    return IRGL_OK;
}

irgl_status irgl_workspace_bytes(irgl_graph g, int32_t kind, int32_t with_parent,
                                 const irgl_config *cfg, size_t *bytes) {
    (void)with_parent;
    if (!g || !bytes) return IRGL_ERR_INVALID_ARGUMENT;
    if (kind != IRGL_KIND_BFS && kind != IRGL_KIND_SSSP) return IRGL_ERR_INVALID_ARGUMENT;
    Cfg c;
    irgl_status st = resolve(g, cfg, &c);
    if (st) return st;
    *bytes = layout(g, kind, c).total;
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
    out->reserved = 0;
    return IRGL_OK;
}

}  // extern "C"
