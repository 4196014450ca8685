/*
 * CPU oracle for the data-driven BFS/SSSP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the package smoke check and the bench's
 * CPU-baseline leg do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition of the result that the paper's
 * worklist BFS (Section 4.1, level-by-level BFS listing: a vertex found
 * while expanding the level-k frontier gets level k+1, starting from the
 * initial worklist [src]) converges to:
 *
 *   level[v] = least number of out-edges on a directed path src -> v,
 *              0xFFFFFFFF when no path exists;
 *   dist[v]  = least sum of uint32 weights (each >= 1) over directed paths
 *              src -> v, 0xFFFFFFFF when no path exists (textbook
 *              single-source shortest paths; the paper states only BFS).
  *
 * Algorithms: a FIFO-queue breadth-first search and a binary-heap Dijkstra
 * with lazy deletion and a 64-bit distance accumulator.  Both are serial and
 * deliberately plain.
 *
 * For the Boruvka workload (the Atomic construct's example, Section 3): the
 * minimum spanning forest of a symmetric weighted CSR by Kruskal's algorithm
 * under the total edge order (w, u, v), which makes the forest unique.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF 0xFFFFFFFFu

/* Serial FIFO breadth-first search over CSR out-edges.
 * level/parent: caller-owned host arrays of length n.
 * parent[src] = src, parent[v] = -1 when unreached, otherwise the vertex
 * that first discovered v.  Returns the number of reached vertices, or -1 on
 * invalid arguments / allocation failure. */
int64_t oracle_bfs(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t src,
                   uint32_t *level, int32_t *parent) {
    if (n <= 0 || src < 0 || src >= n || !row_ptr || !col || !level) return -1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -1;
    for (int32_t v = 0; v < n; ++v) {
        level[v] = ORACLE_INF;
        if (parent) parent[v] = -1;
    }
    int64_t head = 0, tail = 0;
    level[src] = 0;
    if (parent) parent[src] = src;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (level[v] == ORACLE_INF) {
                level[v] = level[u] + 1;
                if (parent) parent[v] = u;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return tail;
}

/* ---- binary min-heap of (distance, vertex) ---------------------------- */
typedef struct {
    uint64_t d;
    int32_t v;
} heap_item;

static void heap_push(heap_item *h, int64_t *size, uint64_t d, int32_t v) {
    int64_t i = (*size)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= d) break;
        h[i] = h[p];
        i = p;
    }
    h[i].d = d;
    h[i].v = v;
}

static heap_item heap_pop(heap_item *h, int64_t *size) {
    heap_item top = h[0];
    heap_item last = h[--(*size)];
    int64_t i = 0, n = *size;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        uint64_t ds = last.d;
        if (l < n && h[l].d < ds) { s = l; ds = h[l].d; }
        if (r < n && h[r].d < ds) { s = r; }
        if (s == i) break;
        h[i] = h[s];
        i = s;
    }
    if (n > 0) h[i] = last;
    return top;
}

/* Binary-heap Dijkstra over CSR out-edges with uint32 weights.
 * dist/parent: caller-owned host arrays of length n.  Distances are
 * accumulated in 64 bits; returns the number of reached vertices, -1 on
 * invalid arguments / allocation failure, -2 if a finite distance does not
 * fit below the 0xFFFFFFFF sentinel (dist is then not written for it). */
int64_t oracle_dijkstra(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        const uint32_t *w, int32_t src, uint32_t *dist, int32_t *parent) {
    if (n <= 0 || src < 0 || src >= n || !row_ptr || !col || !w || !dist) return -1;
    int64_t m = row_ptr[n];
    uint64_t *d64 = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    heap_item *heap = (heap_item *)malloc((size_t)(m + 1) * sizeof(heap_item));
    if (!d64 || !heap) {
        free(d64);
        free(heap);
        return -1;
    }
    const uint64_t UNSEEN = UINT64_MAX;
    for (int32_t v = 0; v < n; ++v) {
        d64[v] = UNSEEN;
        if (parent) parent[v] = -1;
    }
    int64_t hs = 0;
    d64[src] = 0;
    if (parent) parent[src] = src;
    heap_push(heap, &hs, 0, src);
    while (hs > 0) {
        heap_item it = heap_pop(heap, &hs);
        int32_t u = it.v;
        if (it.d > d64[u]) continue; /* stale entry */
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            uint64_t nd = it.d + (uint64_t)w[e];
            if (nd < d64[v]) {
                d64[v] = nd;
                if (parent) parent[v] = u;
                heap_push(heap, &hs, nd, v);
            }
        }
    }
    int64_t reached = 0;
    int overflow = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (d64[v] == UNSEEN) {
            dist[v] = ORACLE_INF;
        } else if (d64[v] >= (uint64_t)ORACLE_INF) {
            overflow = 1;
            dist[v] = ORACLE_INF;
        } else {
            dist[v] = (uint32_t)d64[v];
            ++reached;
        }
    }
    free(d64);
    free(heap);
    return overflow ? -2 : reached;
}

/* Sum of out-degrees of the vertices with level != INF: the number of CSR
 * entries an exact top-down traversal from the source scans. */
int64_t oracle_edges_scanned(int32_t n, const int32_t *row_ptr, const uint32_t *level) {
    int64_t s = 0;
    for (int32_t v = 0; v < n; ++v)
        if (level[v] != ORACLE_INF) s += (int64_t)row_ptr[v + 1] - row_ptr[v];
    return s;
}

/* Distance certificate: checks that d[] (uint32, 0xFFFFFFFF = unreached) is
 * exactly the shortest-path distance vector from src over CSR out-edges with
 * weights w (>= 1; NULL means every weight is 1, i.e. BFS levels), without
 * computing any distance itself.  With weights >= 1 these three conditions
 * hold for exactly one vector:
 *   (i)   d[src] == 0;
 *   (ii)  every edge u -> v with d[u] finite has d[v] finite and
 *         d[v] <= d[u] + w  (so d is at most the true distance);
 *   (iii) every v != src with d[v] finite has an in-edge u -> v with
 *         d[u] + w == d[v]   (so d is at least the true distance: following
 *         such edges backwards strictly decreases d and can only stop at src).
 * One pass over the edges.  Returns 0 when d is certified; otherwise a
 * positive code (1, 2 or 3 for the condition that fails, 4 for a weight of
 * 0) and the offending vertex (or edge source) in *where; -1 on invalid
 * arguments or allocation failure. */
int64_t oracle_certify(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *w, int32_t src,
                       const uint32_t *d, int64_t *where) {
    if (n <= 0 || src < 0 || src >= n || !row_ptr || !col || !d || !where) return -1;
    *where = -1;
    if (d[src] != 0) {
        *where = src;
        return 1;
    }
    unsigned char *tight = (unsigned char *)calloc((size_t)n, 1);
    if (!tight) return -1;
    int64_t code = 0;
    for (int32_t u = 0; u < n && !code; ++u) {
        if (d[u] == ORACLE_INF) continue;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t v = col[e];
            const uint64_t wt = w ? (uint64_t)w[e] : 1u;
            if (wt == 0) {
                code = 4;
                *where = u;
                break;
            }
            const uint64_t cand = (uint64_t)d[u] + wt;
            if (d[v] == ORACLE_INF || (uint64_t)d[v] > cand) {
                code = 2;
                *where = u;
                break;
            }
            if ((uint64_t)d[v] == cand) tight[v] = 1;
        }
    }
    for (int32_t v = 0; v < n && !code; ++v) {
        if (v != src && d[v] != ORACLE_INF && !tight[v]) {
            code = 3;
            *where = v;
        }
    }
    free(tight);
    return code;
}

/* ---- minimum spanning forest ------------------------------------------- */
/*
 * Minimum spanning forest of an undirected graph stored as a symmetric CSR
 * (each edge {u, v} appears as u -> v and v -> u with the same weight).
 * Kruskal's algorithm, written out plainly: list every undirected edge once
 * (as its u < v entry), sort the list by the total order (w, u, v) -- under a
 * total order the minimum forest is unique, so edge sets can be compared --
 * and take each edge whose endpoints are still in different trees of a
 * union-find (path halving, union by size).  Self-loops never join two trees.
 *
 * in_forest: caller-owned uint8[m]; both stored directions of every forest
 * edge are set to 1, the rest to 0.  component: caller-owned int32[n] or
 * NULL; the smallest vertex id of the vertex's tree.  *edges = forest edges.
 * Returns the forest weight, -1 on invalid arguments / allocation failure,
 * -3 when the CSR is not symmetric: the u > v entries, each named by its
 * (v, u), must be exactly the u < v entries with equal weights (as multisets).
 * Sorting both halves by (u, v, w) pairs every edge with its reverse entry.
 */
typedef struct {
    uint32_t w;
    int32_t u, v;
    int64_t e; /* index of the u -> v entry */
    int64_t f; /* index of the matching v -> u entry */
} mst_edge;

/* the total order (w, u, v) */
static int mst_edge_cmp(const void *a, const void *b) {
    const mst_edge *x = (const mst_edge *)a, *y = (const mst_edge *)b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    if (x->u != y->u) return x->u < y->u ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}

/* pairing order of the two halves of a symmetric CSR: (u, v, w, entry); the
   rows' own order makes the u < v half almost sorted already */
static int mst_pair_cmp(const void *a, const void *b) {
    const mst_edge *x = (const mst_edge *)a, *y = (const mst_edge *)b;
    if (x->u != y->u) return x->u < y->u ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    if (x->e != y->e) return x->e < y->e ? -1 : 1;
    return 0;
}

static int32_t uf_find(int32_t *parent, int32_t x) {
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

int64_t oracle_kruskal(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                       uint8_t *in_forest, int32_t *component, int64_t *edges) {
    if (n <= 0 || !row_ptr || !col || !w || !in_forest || !edges) return -1;
    const int64_t m = row_ptr[n];
    int64_t cnt = 0, rcnt = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            if (u < col[e]) ++cnt;
            if (u > col[e]) ++rcnt;
        }
    if (cnt != rcnt) return -3;
    mst_edge *list = (mst_edge *)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(mst_edge));
    mst_edge *back = (mst_edge *)malloc((size_t)(cnt > 0 ? cnt : 1) * sizeof(mst_edge));
    int32_t *parent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *size = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!list || !back || !parent || !size) {
        free(list);
        free(back);
        free(parent);
        free(size);
        return -1;
    }
    /* list: the u < v entries; back: the u > v entries, named by (v, u) */
    int64_t k = 0, r = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            if (u < col[e]) {
                list[k].w = w[e];
                list[k].u = u;
                list[k].v = col[e];
                list[k].e = e;
                ++k;
            } else if (u > col[e]) {
                back[r].w = w[e];
                back[r].u = col[e];
                back[r].v = u;
                back[r].e = e;
                ++r;
            }
        }
    /* symmetric input: sorted the same way, the two halves agree entry by
       entry, and each edge learns its reverse entry */
    qsort(list, (size_t)cnt, sizeof(mst_edge), mst_pair_cmp);
    qsort(back, (size_t)cnt, sizeof(mst_edge), mst_pair_cmp);
    for (int64_t i = 0; i < cnt; ++i) {
        if (list[i].u != back[i].u || list[i].v != back[i].v || list[i].w != back[i].w) {
            free(list);
            free(back);
            free(parent);
            free(size);
            return -3;
        }
        list[i].f = back[i].e;
    }
    free(back);
    qsort(list, (size_t)cnt, sizeof(mst_edge), mst_edge_cmp);
    for (int32_t v = 0; v < n; ++v) {
        parent[v] = v;
        size[v] = 1;
    }
    memset(in_forest, 0, (size_t)m);
    int64_t total = 0, taken = 0;
    for (int64_t i = 0; i < cnt; ++i) {
        int32_t a = uf_find(parent, list[i].u), b = uf_find(parent, list[i].v);
        if (a == b) continue;
        if (size[a] < size[b]) {
            int32_t t = a;
            a = b;
            b = t;
        }
        parent[b] = a;
        size[a] += size[b];
        in_forest[list[i].e] = 1;
        in_forest[list[i].f] = 1;
        total += list[i].w;
        ++taken;
    }
    if (component) {
        /* the smallest vertex id of each tree, through its root */
        for (int32_t v = 0; v < n; ++v) size[v] = n;
        for (int32_t v = 0; v < n; ++v) {
            int32_t r = uf_find(parent, v);
            if (v < size[r]) size[r] = v;
        }
        for (int32_t v = 0; v < n; ++v) component[v] = size[uf_find(parent, v)];
    }
    free(list);
    free(parent);
    free(size);
    *edges = taken;
    return total;
}
