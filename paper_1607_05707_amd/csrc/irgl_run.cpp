// irgl_run: native command-line runner of the C ABI (no Python in the
// process), for timing and profiling BFS/SSSP queries on a CSR file written
// by paper_1607_05707_amd.workloads.
//
//   irgl_run FILE [--kinds bfs,sssp] [--sources K] [--reps R] [--warmup W]
//                 [--block B] [--mode 0|1] [--t-grid T] [--t-bitmap T]
//                 [--do-alpha A] [--do-beta B] [--delta D] [--calibrate MB] [--reorder 0|1]
//                 [--set-delta D] [--maps FILE]
//
// --calibrate MB first copies MB megabytes device-to-device once (a plain
// copy of known traffic, to scale hardware byte counters).  --set-delta D
// changes the graph's default SSSP near/far step after the upload (on a
// relabelled weighted graph it also rebuilds the light/heavy partition).
// --maps FILE copies the process's memory map (/proc/self/maps) to FILE
// just before main returns, so that an address reported by a fault after
// main (in a library destructor at exit) can be attributed to a library.
//
// FILE may also be a mesh file written by paper_1607_05707_amd.meshgen: the
// runner then refines it (irgl_dmr_refine) `--reps` times after `--warmup`
// untimed runs, each on a fresh copy, and prints the mean time and the
// statistics of the last run.
//
// Prints one line per kind: queries, mean microseconds per query (hipEvent
// pairs around each call on one stream) and GTEPS (out-degree sum of the
// vertices a BFS from each source reaches / time).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "irgl.h"

#define CK(x)                                                                          \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)
#define CI(x)                                                                          \
    do {                                                                               \
        irgl_status s_ = (x);                                                          \
        if (s_ != IRGL_OK) {                                                           \
            std::fprintf(stderr, "irgl error %s at line %d\n", irgl_status_string(s_), __LINE__); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

static void write_maps(const std::string &path) {
    if (path.empty()) return;
    FILE *in = std::fopen("/proc/self/maps", "r");
    FILE *out = std::fopen(path.c_str(), "w");
    if (in && out) {
        char buf[4096];
        size_t k;
        while ((k = std::fread(buf, 1, sizeof(buf), in)) > 0) std::fwrite(buf, 1, k, out);
    }
    if (in) std::fclose(in);
    if (out) std::fclose(out);
}

// Delaunay mesh refinement of a mesh file, `reps` timed runs (each on a fresh
// copy of the input) after `warmup` untimed ones.
static int run_mesh(const char *path, int reps, int warmup, const std::string &maps_out) {
    FILE *f = std::fopen(path, "rb");
    char magic[8];
    int64_t hdr[4];
    if (!f || std::fread(magic, 1, 8, f) != 8 || std::fread(hdr, 8, 4, f) != 4) {
        std::fprintf(stderr, "bad mesh file\n");
        return 1;
    }
    const int64_t npts = hdr[0], ntri = hdr[1], pcap = hdr[2], tcap = hdr[3];
    if (npts < 3 || ntri < 1 || pcap < npts || tcap < ntri || pcap >= (1 << 30) || tcap >= (1 << 30)) {
        std::fprintf(stderr, "bad mesh sizes\n");
        return 1;
    }
    std::vector<double> pts(static_cast<size_t>(pcap) * 2);
    std::vector<int32_t> tri(static_cast<size_t>(tcap) * 4), nbr(static_cast<size_t>(tcap) * 4);
    const bool ok = std::fread(pts.data(), 8, pts.size(), f) == pts.size() &&
                    std::fread(tri.data(), 4, tri.size(), f) == tri.size() &&
                    std::fread(nbr.data(), 4, nbr.size(), f) == nbr.size();
    std::fclose(f);
    if (!ok) {
        std::fprintf(stderr, "short mesh file\n");
        return 1;
    }
    double *d_pts;
    int32_t *d_tri, *d_nbr;
    CK(hipMalloc(&d_pts, pts.size() * 8));
    CK(hipMalloc(&d_tri, tri.size() * 4));
    CK(hipMalloc(&d_nbr, nbr.size() * 4));
    irgl_mesh m{d_pts, d_tri, d_nbr, static_cast<int32_t>(npts), static_cast<int32_t>(ntri),
                static_cast<int32_t>(pcap), static_cast<int32_t>(tcap)};
    size_t wsb = 0;
    CI(irgl_dmr_workspace_bytes(&m, &wsb));
    void *ws;
    CK(hipMalloc(&ws, wsb));
    irgl_dmr_stats *d_stats;
    CK(hipMalloc(&d_stats, sizeof(irgl_dmr_stats)));
    hipStream_t s;
    CK(hipStreamCreate(&s));
    hipEvent_t a, b;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    double tot_ms = 0;
    irgl_dmr_stats st{};
    for (int r = 0; r < warmup + reps; ++r) {
        CK(hipMemcpy(d_pts, pts.data(), pts.size() * 8, hipMemcpyHostToDevice));
        CK(hipMemcpy(d_tri, tri.data(), tri.size() * 4, hipMemcpyHostToDevice));
        CK(hipMemcpy(d_nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice));
        CK(hipEventRecord(a, s));
        CI(irgl_dmr_refine(&m, ws, wsb, nullptr, s, d_stats));
        CK(hipEventRecord(b, s));
        CK(hipStreamSynchronize(s));
        CK(hipMemcpy(&st, d_stats, sizeof(st), hipMemcpyDeviceToHost));
        if (st.status) {
            std::fprintf(stderr, "dmr: %s\n", irgl_status_string(st.status));
            return 1;
        }
        float ms;
        CK(hipEventElapsedTime(&ms, a, b));
        if (r >= warmup) tot_ms += ms;
    }
    std::printf("dmr runs=%d mean_ms=%.3f points=%d triangles=%d inserted=%u splits=%u invocations=%u "
                "rounds=%u conflicts=%llu final_bad=%u grid=%dx%d\n", reps, tot_ms / (reps > 0 ? reps : 1),
                st.npts, st.ntri, st.inserted, st.splits, st.invocations, st.rounds,
                static_cast<unsigned long long>(st.conflicts), st.final_bad, st.grid, st.block);
    CK(hipEventDestroy(a));
    CK(hipEventDestroy(b));
    CK(hipStreamDestroy(s));
    CK(hipFree(d_stats));
    CK(hipFree(ws));
    CK(hipFree(d_pts));
    CK(hipFree(d_tri));
    CK(hipFree(d_nbr));
    CI(irgl_shutdown());
    write_maps(maps_out);
    std::printf("runner done\n");
    std::fflush(stdout);
    return 0;
}

int main(int argc, char **argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: %s FILE [options]\n", argv[0]);
        return 2;
    }
    std::string kinds = "bfs,sssp";
    int nsrc = 8, reps = 1, warmup = 1;
    long calib_mb = 0;
    int reorder = 0;
    uint32_t set_delta = 0;  // irgl_graph_set_delta after the upload (0: keep the default step)
    std::string maps_out;
    irgl_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    for (int i = 2; i + 1 < argc; i += 2) {
        std::string k = argv[i];
        const char *v = argv[i + 1];
        if (k == "--kinds") kinds = v;
        else if (k == "--sources") nsrc = std::atoi(v);
        else if (k == "--reps") reps = std::atoi(v);
        else if (k == "--warmup") warmup = std::atoi(v);
        else if (k == "--block") cfg.block = std::atoi(v);
        else if (k == "--mode") cfg.mode = std::atoi(v);
        else if (k == "--t-grid") cfg.t_grid = std::atoi(v);
        else if (k == "--t-bitmap") cfg.t_bitmap = static_cast<uint32_t>(std::strtoul(v, nullptr, 0));
        else if (k == "--do-alpha") cfg.do_alpha = static_cast<uint32_t>(std::strtoul(v, nullptr, 0));
        else if (k == "--do-beta") cfg.do_beta = static_cast<uint32_t>(std::strtoul(v, nullptr, 0));
        else if (k == "--delta") cfg.delta = static_cast<uint32_t>(std::strtoul(v, nullptr, 0));
        else if (k == "--reorder") reorder = std::atoi(v);
        else if (k == "--set-delta") set_delta = static_cast<uint32_t>(std::strtoul(v, nullptr, 0));
        else if (k == "--maps") maps_out = v;
        else if (k == "--calibrate") calib_mb = std::atol(v);
        else {
            std::fprintf(stderr, "unknown option %s\n", k.c_str());
            return 2;
        }
    }
    {
        // a mesh file (meshgen.py): Delaunay refinement instead of queries
        FILE *mf = std::fopen(argv[1], "rb");
        char mg[8] = {0};
        const bool is_mesh = mf && std::fread(mg, 1, 8, mf) == 8 && std::memcmp(mg, "IRGLMSH1", 8) == 0;
        if (mf) std::fclose(mf);
        if (is_mesh) return run_mesh(argv[1], reps, warmup, maps_out);
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) {
        std::perror(argv[1]);
        return 1;
    }
    char magic[8];
    int64_t hdr[4];
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "IRGLCSR1", 8) != 0 ||
        std::fread(hdr, 8, 4, f) != 4) {
        std::fprintf(stderr, "bad file header\n");
        return 1;
    }
    const int64_t n = hdr[0], m = hdr[1], has_w = hdr[2] & 1, symmetric = (hdr[2] >> 1) & 1, ns = hdr[3];
    if (n <= 0 || n >= (int64_t(1) << 31) || m < 0 || m >= (int64_t(1) << 31) || ns <= 0) {
        std::fprintf(stderr, "bad sizes\n");
        return 1;
    }
    std::vector<int32_t> rp(n + 1), col(m), src(ns);
    std::vector<uint32_t> w(has_w ? m : 0);
    bool ok = std::fread(rp.data(), 4, n + 1, f) == static_cast<size_t>(n + 1) &&
              std::fread(col.data(), 4, m, f) == static_cast<size_t>(m) &&
              (!has_w || std::fread(w.data(), 4, m, f) == static_cast<size_t>(m)) &&
              std::fread(src.data(), 4, ns, f) == static_cast<size_t>(ns);
    std::fclose(f);
    if (!ok) {
        std::fprintf(stderr, "short file\n");
        return 1;
    }
    if (nsrc > ns) nsrc = static_cast<int>(ns);
    if (calib_mb > 0) {
        const size_t bytes = static_cast<size_t>(calib_mb) << 20;
        void *a, *b;
        CK(hipMalloc(&a, bytes));
        CK(hipMalloc(&b, bytes));
        CK(hipMemset(a, 1, bytes));
        CK(hipDeviceSynchronize());
        CK(hipMemcpy(b, a, bytes, hipMemcpyDeviceToDevice));
        CK(hipDeviceSynchronize());
        std::printf("calibration copy: %zu bytes read + %zu bytes written\n", bytes, bytes);
        CK(hipFree(a));
        CK(hipFree(b));
    }

    int32_t *d_rp, *d_col, *d_out;
    uint32_t *d_w = nullptr;
    CK(hipMalloc(&d_rp, (n + 1) * 4));
    CK(hipMalloc(&d_col, m * 4 + 4));
    CK(hipMalloc(&d_out, n * 4));
    CK(hipMemcpy(d_rp, rp.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_col, col.data(), m * 4, hipMemcpyHostToDevice));
    if (has_w) {
        CK(hipMalloc(&d_w, m * 4 + 4));
        CK(hipMemcpy(d_w, w.data(), m * 4, hipMemcpyHostToDevice));
    }
    irgl_csr csr{static_cast<int32_t>(n), m, d_rp, d_col, d_w, IRGL_VALIDATE | (symmetric ? IRGL_SYMMETRIC : 0u)};
    irgl_graph g;
    void *store = nullptr;
    if (reorder) {
        size_t sb = 0;
        CI(irgl_reorder_bytes(csr.n, csr.m, d_w != nullptr, &sb));
        CK(hipMalloc(&store, sb));
        CI(irgl_graph_upload_reordered(&csr, store, sb, &g));
    } else {
        CI(irgl_graph_upload(&csr, &g));
    }
    if (set_delta) CI(irgl_graph_set_delta(g, set_delta));
    uint32_t qdelta = 0;
    CI(irgl_graph_default_delta(g, &qdelta));
    std::printf("default near/far step %u\n", qdelta);
    irgl_stats *d_stats;
    CK(hipMalloc(&d_stats, sizeof(irgl_stats)));
    hipStream_t s;
    CK(hipStreamCreate(&s));

    std::vector<uint64_t> mcc(nsrc, 0);
    for (int kind : {IRGL_KIND_BFS, IRGL_KIND_SSSP}) {
        const char *name = kind == IRGL_KIND_BFS ? "bfs" : "sssp";
        if (kinds.find(name) == std::string::npos && kind == IRGL_KIND_SSSP) continue;
        if (kind == IRGL_KIND_SSSP && !has_w) continue;
        size_t wsb = 0;
        CI(irgl_workspace_bytes(g, kind, 0, &cfg, &wsb));
        void *ws;
        CK(hipMalloc(&ws, wsb));
        auto run = [&](int32_t sv) {
            return kind == IRGL_KIND_BFS ? irgl_bfs(g, sv, reinterpret_cast<uint32_t *>(d_out), nullptr, ws,
                                                    wsb, s, d_stats, &cfg)
                                         : irgl_sssp(g, sv, reinterpret_cast<uint32_t *>(d_out), nullptr, ws,
                                                     wsb, s, d_stats, &cfg);
        };
        if (kind == IRGL_KIND_BFS) {  // numerator: out-degree sum of the reached vertices
            for (int i = 0; i < nsrc; ++i) {
                CI(run(src[i]));
                irgl_stats st;
                CI(irgl_query_status(ws, s, &st));
                if (st.status) {
                    std::fprintf(stderr, "bfs from %d: %s\n", src[i], irgl_status_string(st.status));
                    return 1;
                }
                mcc[i] = st.frontier_edges;
            }
        }
        for (int r = 0; r < warmup; ++r)
            for (int i = 0; i < nsrc; ++i) CI(run(src[i]));
        std::vector<hipEvent_t> ev(2 * nsrc * reps);
        for (auto &e : ev) CK(hipEventCreate(&e));
        int k = 0;
        for (int r = 0; r < reps; ++r)
            for (int i = 0; i < nsrc; ++i) {
                CK(hipEventRecord(ev[k++], s));
                CI(run(src[i]));
                CK(hipEventRecord(ev[k++], s));
            }
        CK(hipStreamSynchronize(s));
        irgl_stats st;
        CI(irgl_query_status(ws, s, &st));
        // work of one more (untimed) pass: CSR entries scanned per reached edge
        double scanned = 0, pulls = 0;
        for (int i = 0; i < nsrc; ++i) {
            CI(run(src[i]));
            irgl_stats sq;
            CI(irgl_query_status(ws, s, &sq));
            if (sq.status) {
                std::fprintf(stderr, "%s from %d: %s\n", name, src[i], irgl_status_string(sq.status));
                return 1;
            }
            scanned += static_cast<double>(sq.edges);
            pulls += sq.heavy_pulls;
        }
        double mcc_sum = 0;
        for (int i = 0; i < nsrc; ++i) mcc_sum += static_cast<double>(mcc[i]);
        double tot_ms = 0, edges = 0;
        for (int q = 0; q < nsrc * reps; ++q) {
            float ms;
            CK(hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]));
            tot_ms += ms;
            edges += static_cast<double>(mcc[q % nsrc]);
        }
        std::printf("%s queries=%d mean_us=%.1f gteps=%.3f status=%d iterations=%u grid=%dx%d "
                    "scans_per_edge=%.3f heavy_pulls=%.2f\n", name, nsrc * reps, 1e3 * tot_ms / (nsrc * reps),
                    edges / (tot_ms * 1e-3) / 1e9, st.status, st.iterations, st.grid, st.block,
                    mcc_sum > 0 ? scanned / mcc_sum : 0.0, nsrc > 0 ? pulls / nsrc : 0.0);
        std::fflush(stdout);
        for (auto &e : ev) CK(hipEventDestroy(e));
        CK(hipFree(ws));
    }
    CI(irgl_graph_free(g));
    if (store) CK(hipFree(store));
    CK(hipStreamDestroy(s));
    CK(hipFree(d_stats));
    CK(hipFree(d_rp));
    CK(hipFree(d_col));
    CK(hipFree(d_out));
    if (d_w) CK(hipFree(d_w));
    CI(irgl_shutdown());
    write_maps(maps_out);
    std::printf("runner done\n");
    std::fflush(stdout);
    return 0;
}
