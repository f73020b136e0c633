/*
 * oracle.c -- CPU reference results for SSSP, BFS and connected components.
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  Plain sequential C; shares nothing with the
 * GPU library.  See oracle.h for the definitions computed and the argument
 * and error conventions.
 *
 * Parity pinning: each routine here is checked by the test suite against
 * routines outside this file (scipy.sparse.csgraph), against closed forms
 * (paths, grids, complete digraphs, stars, disjoint blocks) and against
 * hand-derived fixtures; the brute-force routines and the certificates in
 * this file are pinned the same way.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

#define INF64 ((int64_t)1 << 62)

/* Shared argument check: CSR shape, column range, optional weight sign. */
static int valid_csr(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w) {
    if (n < 1 || !row_ptr) return 0;
    if (row_ptr[0] != 0) return 0;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return 0;
    int64_t m = row_ptr[n];
    if (m > 0 && !col) return 0;
    for (int64_t e = 0; e < m; ++e) {
        if (col[e] < 0 || col[e] >= n) return 0;
        if (w && w[e] < 0) return 0;
    }
    return 1;
}

static int32_t clamp_inf(int64_t d) { return d >= ORACLE_INF ? ORACLE_INF : (int32_t)d; }

/* ------------------------------------------------------------ SSSP ----- */
/* The paper's SSSP (Algorithms 1 and 2) lowers t.dist to p.dist + weight
 * along every edge p -> t until nothing changes.  With non-negative weights
 * the fixpoint is the shortest-path distance, which Dijkstra's algorithm
 * computes directly. */

typedef struct {
    int64_t d;
    int32_t v;
} heap_item;

typedef struct {
    heap_item* a;
    int64_t size, cap;
} heap_t;

static int heap_push(heap_t* h, int64_t d, int32_t v) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        heap_item* na = (heap_item*)realloc(h->a, (size_t)nc * sizeof(heap_item));
        if (!na) return -3;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    while (i > 0) {
        int64_t parent = (i - 1) / 2;
        if (h->a[parent].d <= d) break;
        h->a[i] = h->a[parent];
        i = parent;
    }
    h->a[i].d = d;
    h->a[i].v = v;
    return 0;
}

static heap_item heap_pop(heap_t* h) {
    heap_item top = h->a[0];
    heap_item last = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, small = i;
        int64_t small_d = last.d;
        if (l < h->size && h->a[l].d < small_d) {
            small = l;
            small_d = h->a[l].d;
        }
        if (r < h->size && h->a[r].d < small_d) small = r;
        if (small == i) break;
        h->a[i] = h->a[small];
        i = small;
    }
    if (h->size > 0) h->a[i] = last;
    return top;
}

int oracle_sssp(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                int32_t source, int32_t* dist) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !dist || source < 0 || source >= n) return -1;
    int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!D) return -3;
    for (int32_t v = 0; v < n; ++v) D[v] = INF64;
    heap_t h = {NULL, 0, 0};
    D[source] = 0;
    int rc = heap_push(&h, 0, source);
    while (rc == 0 && h.size > 0) {
        heap_item it = heap_pop(&h);
        int32_t u = it.v;
        if (it.d > D[u]) continue; /* stale entry */
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            int64_t nd = it.d + (int64_t)w[e];
            if (nd < D[v]) {
                D[v] = nd;
                rc = heap_push(&h, nd, v);
                if (rc) break;
            }
        }
    }
    if (rc == 0)
        for (int32_t v = 0; v < n; ++v) dist[v] = clamp_inf(D[v]);
    free(h.a);
    free(D);
    return rc;
}

/* ------------------------------------------------------------- BFS ----- */
/* Algorithm 3 assigns level lev+1 to every unvisited out-neighbour of a
 * level-lev vertex, level by level; its fixpoint is the hop distance, which
 * a FIFO breadth-first search computes directly. */

int oracle_bfs(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t source,
               int32_t* dist) {
    if (!valid_csr(n, row_ptr, col, NULL) || !dist || source < 0 || source >= n) return -1;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -3;
    for (int32_t v = 0; v < n; ++v) dist[v] = ORACLE_INF;
    int64_t head = 0, tail = 0;
    dist[source] = 0;
    queue[tail++] = source;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (dist[v] == ORACLE_INF) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* -------------------------------------------------------------- CC ----- */
/* Connected components (Sec. 4.1 names the algorithm; Sec. 2 describes the
 * DSL's Set type as a union-find structure).  Components of the graph with
 * each edge taken in both directions; label = smallest member id. */

static int32_t uf_find(int32_t* parent, int32_t x) {
    while (parent[x] != x) {
        parent[x] = parent[parent[x]]; /* path halving */
        x = parent[x];
    }
    return x;
}

int oracle_cc(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* label) {
    if (!valid_csr(n, row_ptr, col, NULL) || !label) return -1;
    int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* size = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* minid = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!parent || !size || !minid) {
        free(parent);
        free(size);
        free(minid);
        return -3;
    }
    for (int32_t v = 0; v < n; ++v) {
        parent[v] = v;
        size[v] = 1;
    }
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t a = uf_find(parent, u), b = uf_find(parent, col[e]);
            if (a == b) continue;
            if (size[a] < size[b]) {
                int32_t t = a;
                a = b;
                b = t;
            }
            parent[b] = a; /* union by size */
            size[a] += size[b];
        }
    }
    for (int32_t v = 0; v < n; ++v) minid[v] = n;
    for (int32_t v = 0; v < n; ++v) {
        int32_t r = uf_find(parent, v);
        if (v < minid[r]) minid[r] = v;
    }
    for (int32_t v = 0; v < n; ++v) label[v] = minid[uf_find(parent, v)];
    free(parent);
    free(size);
    free(minid);
    return 0;
}

/* ------------------------------------------------------------- MST ----- */
/* Minimum spanning forest: the fourth algorithm of the evaluation (Sec. 4.1,
 * Table 3); the DSL's Set type is a union-find structure (Sec. 2).  Every
 * stored edge e = (u, col[e]) with weight w[e] is taken as an undirected
 * edge with key (w[e], e), compared as the 64-bit number w[e] * 2^32 + e.
 * Keys are distinct, so the spanning forest of least key is unique; a
 * self-loop never belongs to it.  Kruskal's algorithm: edges in increasing
 * key order; an edge joins the forest when its ends lie in different sets. */

static uint64_t msf_key(const int32_t* w, int64_t e) { return ((uint64_t)w[e] << 32) | (uint64_t)e; }

static int cmp_u64(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

static int32_t* edge_sources(int32_t n, const int32_t* row_ptr) {
    int32_t* src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(row_ptr[n] + 1));
    if (!src) return NULL;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) src[e] = u;
    return src;
}

int oracle_msf(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
               uint8_t* in_msf, int64_t* total_weight) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !in_msf) return -1;
    const int64_t m = row_ptr[n];
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m + 1));
    int32_t* src = edge_sources(n, row_ptr);
    int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* size = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!keys || !src || !parent || !size) {
        free(keys);
        free(src);
        free(parent);
        free(size);
        return -3;
    }
    for (int64_t e = 0; e < m; ++e) {
        keys[e] = msf_key(w, e);
        in_msf[e] = 0;
    }
    qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);
    for (int32_t v = 0; v < n; ++v) {
        parent[v] = v;
        size[v] = 1;
    }
    int64_t total = 0;
    for (int64_t i = 0; i < m; ++i) {
        const int64_t e = (int64_t)(keys[i] & 0xffffffffu);
        int32_t a = uf_find(parent, src[e]), b = uf_find(parent, col[e]);
        if (a == b) continue;
        if (size[a] < size[b]) {
            int32_t t = a;
            a = b;
            b = t;
        }
        parent[b] = a;
        size[a] += size[b];
        in_msf[e] = 1;
        total += w[e];
    }
    if (total_weight) *total_weight = total;
    free(keys);
    free(src);
    free(parent);
    free(size);
    return 0;
}

/* Brute force (n <= 10, m <= 20, weights < 2^24): among all edge subsets
 * with n - (number of components) edges and no cycle, the one of least
 * summed key (exact, 128-bit). */
int oracle_msf_brute(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                     uint8_t* in_msf) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !in_msf || n > 10 || row_ptr[n] > 20) return -1;
    const int32_t m = row_ptr[n];
    int32_t src[20], parent[10];
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) src[e] = u;
    for (int32_t e = 0; e < m; ++e)
        if (w[e] >= (1 << 24)) return -1;
    /* components of the whole graph */
    for (int32_t v = 0; v < n; ++v) parent[v] = v;
    int32_t comps = n;
    for (int32_t e = 0; e < m; ++e) {
        int32_t a = uf_find(parent, src[e]), b = uf_find(parent, col[e]);
        if (a != b) {
            parent[a] = b;
            --comps;
        }
    }
    const int32_t want = n - comps;
    unsigned __int128 best = 0;
    int64_t best_set = -1;
    for (int64_t set = 0; set < ((int64_t)1 << m); ++set) {
        if (__builtin_popcountll((unsigned long long)set) != want) continue;
        for (int32_t v = 0; v < n; ++v) parent[v] = v;
        int ok = 1;
        unsigned __int128 sum = 0;
        for (int32_t e = 0; e < m && ok; ++e) {
            if (!((set >> e) & 1)) continue;
            int32_t a = uf_find(parent, src[e]), b = uf_find(parent, col[e]);
            if (a == b) ok = 0;
            else parent[a] = b;
            sum += msf_key(w, e);
        }
        if (ok && (best_set < 0 || sum < best)) {
            best = sum;
            best_set = set;
        }
    }
    for (int32_t e = 0; e < m; ++e) in_msf[e] = best_set >= 0 ? (uint8_t)((best_set >> e) & 1) : 0;
    return 0;
}

/* ----------------------------------------------------- brute force ----- */

#define BRUTE_MAX_N 512

int oracle_sssp_floyd_warshall(int32_t n, const int32_t* row_ptr, const int32_t* col,
                               const int32_t* w, int32_t source, int32_t* dist) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !dist || source < 0 || source >= n ||
        n > BRUTE_MAX_N)
        return -1;
    int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * (size_t)n);
    if (!D) return -3;
    for (int64_t i = 0; i < (int64_t)n * n; ++i) D[i] = INF64;
    for (int32_t i = 0; i < n; ++i) D[(int64_t)i * n + i] = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t* cell = &D[(int64_t)u * n + col[e]];
            if ((int64_t)w[e] < *cell) *cell = w[e];
        }
    for (int32_t k = 0; k < n; ++k)
        for (int32_t i = 0; i < n; ++i) {
            int64_t dik = D[(int64_t)i * n + k];
            if (dik == INF64) continue;
            for (int32_t j = 0; j < n; ++j) {
                int64_t dkj = D[(int64_t)k * n + j];
                if (dkj != INF64 && dik + dkj < D[(int64_t)i * n + j])
                    D[(int64_t)i * n + j] = dik + dkj;
            }
        }
    for (int32_t v = 0; v < n; ++v) dist[v] = clamp_inf(D[(int64_t)source * n + v]);
    free(D);
    return 0;
}

int oracle_sssp_bellman_ford(int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* w, int32_t source, int32_t* dist) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !dist || source < 0 || source >= n ||
        n > BRUTE_MAX_N)
        return -1;
    int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!D) return -3;
    for (int32_t v = 0; v < n; ++v) D[v] = INF64;
    D[source] = 0;
    /* n-1 rounds over every edge; a shortest path has at most n-1 edges */
    for (int32_t round = 0; round + 1 < n; ++round) {
        int changed = 0;
        for (int32_t u = 0; u < n; ++u) {
            if (D[u] == INF64) continue;
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (D[u] + w[e] < D[col[e]]) {
                    D[col[e]] = D[u] + w[e];
                    changed = 1;
                }
        }
        if (!changed) break;
    }
    for (int32_t v = 0; v < n; ++v) dist[v] = clamp_inf(D[v]);
    free(D);
    return 0;
}

int oracle_cc_warshall(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* label) {
    if (!valid_csr(n, row_ptr, col, NULL) || !label || n > BRUTE_MAX_N) return -1;
    unsigned char* R = (unsigned char*)calloc((size_t)n * (size_t)n, 1);
    if (!R) return -3;
    for (int32_t i = 0; i < n; ++i) R[(int64_t)i * n + i] = 1;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            R[(int64_t)u * n + col[e]] = 1;
            R[(int64_t)col[e] * n + u] = 1;
        }
    /* Warshall's transitive closure */
    for (int32_t k = 0; k < n; ++k)
        for (int32_t i = 0; i < n; ++i)
            if (R[(int64_t)i * n + k])
                for (int32_t j = 0; j < n; ++j)
                    if (R[(int64_t)k * n + j]) R[(int64_t)i * n + j] = 1;
    for (int32_t v = 0; v < n; ++v) {
        int32_t j = 0;
        while (!R[(int64_t)v * n + j]) ++j;
        label[v] = j;
    }
    free(R);
    return 0;
}

/* ----------------------------------------------------- certificates ---- */

int oracle_check_sssp(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                      int32_t source, const int32_t* dist) {
    if (!valid_csr(n, row_ptr, col, w) || !dist || source < 0 || source >= n) return -1;
    if (dist[source] != 0) return 1;
    for (int32_t v = 0; v < n; ++v)
        if (dist[v] < 0) return 2;
    /* feasibility: no edge can still lower its head */
    for (int32_t u = 0; u < n; ++u) {
        if (dist[u] == ORACLE_INF) continue;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t cand = (int64_t)dist[u] + (w ? w[e] : 1);
            if (cand < (int64_t)dist[col[e]]) return 3;
        }
    }
    /* tightness: the tight edges from the source reach every finite vertex
     * and only those (feasible + reached by a tight path => exact) */
    unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return -3;
    }
    int64_t head = 0, tail = 0;
    seen[source] = 1;
    queue[tail++] = source;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (seen[v] || dist[v] == ORACLE_INF) continue;
            if ((int64_t)dist[u] + (w ? w[e] : 1) == (int64_t)dist[v]) {
                seen[v] = 1;
                queue[tail++] = v;
            }
        }
    }
    int rc = 0;
    for (int32_t v = 0; v < n && !rc; ++v)
        if ((dist[v] != ORACLE_INF) != (seen[v] != 0)) rc = 4;
    free(seen);
    free(queue);
    return rc;
}

int oracle_check_cc(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* label) {
    if (!valid_csr(n, row_ptr, col, NULL) || !label) return -1;
    for (int32_t v = 0; v < n; ++v)
        if (label[v] < 0 || label[v] > v) return 1;
    for (int32_t v = 0; v < n; ++v)
        if (label[label[v]] != label[v]) return 2;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (label[u] != label[col[e]]) return 3;
    /* undirected adjacency: out-edges plus reversed edges */
    int64_t m = row_ptr[n];
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!start || !adj || !seen || !queue) {
        free(start);
        free(adj);
        free(seen);
        free(queue);
        return -3;
    }
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            start[u + 1]++;
            start[col[e] + 1]++;
        }
    for (int32_t v = 0; v < n; ++v) start[v + 1] += start[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!fill) {
        free(start);
        free(adj);
        free(seen);
        free(queue);
        return -3;
    }
    memcpy(fill, start, sizeof(int64_t) * (size_t)n);
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            adj[fill[u]++] = col[e];
            adj[fill[col[e]]++] = u;
        }
    int64_t components = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (seen[s]) continue;
        ++components;
        int64_t head = 0, tail = 0;
        seen[s] = 1;
        queue[tail++] = s;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t k = start[u]; k < start[u + 1]; ++k)
                if (!seen[adj[k]]) {
                    seen[adj[k]] = 1;
                    queue[tail++] = adj[k];
                }
        }
    }
    /* a label is its own fixed point, so distinct labels are counted by
     * the vertices that label themselves */
    int64_t distinct = 0;
    for (int32_t v = 0; v < n; ++v)
        if (label[v] == v) ++distinct;
    free(start);
    free(adj);
    free(seen);
    free(queue);
    free(fill);
    return distinct == components ? 0 : 4;
}

/* MSF certificate.  The selected edges must form a forest (no self-loop, no
 * cycle: 1), span every component of the graph (as many edges as vertices
 * minus components, components counted by a breadth-first search over the
 * undirected adjacency: 2), and every edge left out must close a cycle whose
 * other edges all have smaller keys (the cycle property: 3).  Together these
 * hold for exactly one edge set, the minimum spanning forest.  Path maxima
 * come from binary lifting over each tree rooted by a breadth-first search. */
int oracle_check_msf(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                     const uint8_t* in_msf) {
    if (!valid_csr(n, row_ptr, col, w) || !w || !in_msf) return -1;
    const int64_t m = row_ptr[n];
    int rc = 0;
    int levels = 1;
    while (((int64_t)1 << levels) < n) ++levels;
    int32_t* src = edge_sources(n, row_ptr);
    int32_t* uf = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int64_t* adj_e = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* depth = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* up = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * (size_t)levels);
    uint64_t* mx = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n * (size_t)levels);
    if (!src || !uf || !start || !fill || !adj || !adj_e || !queue || !depth || !up || !mx) {
        rc = -3;
        goto done;
    }
    /* 1: a forest */
    for (int32_t v = 0; v < n; ++v) uf[v] = v;
    int64_t chosen = 0;
    for (int64_t e = 0; e < m && !rc; ++e) {
        if (!in_msf[e]) continue;
        ++chosen;
        const int32_t a = uf_find(uf, src[e]), b = uf_find(uf, col[e]);
        if (a == b) rc = 1;
        else uf[a] = b;
    }
    if (rc) goto done;
    /* 2: spanning -- components of the whole graph by BFS */
    for (int64_t e = 0; e < m; ++e) {
        start[src[e] + 1]++;
        start[col[e] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) start[v + 1] += start[v];
    memcpy(fill, start, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) {
        adj[fill[src[e]]] = col[e];
        adj_e[fill[src[e]]++] = e;
        adj[fill[col[e]]] = src[e];
        adj_e[fill[col[e]]++] = e;
    }
    int64_t comps = 0;
    for (int32_t v = 0; v < n; ++v) depth[v] = -1;
    for (int32_t s0 = 0; s0 < n; ++s0) {
        if (depth[s0] >= 0) continue;
        ++comps;
        int64_t head = 0, tail = 0;
        depth[s0] = 0;
        queue[tail++] = s0;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int64_t k = start[u]; k < start[u + 1]; ++k)
                if (depth[adj[k]] < 0) {
                    depth[adj[k]] = 0;
                    queue[tail++] = adj[k];
                }
        }
    }
    if (chosen != (int64_t)n - comps) {
        rc = 2;
        goto done;
    }
    /* 3: root every tree of the forest, then check each edge left out */
    for (int32_t v = 0; v < n; ++v) depth[v] = -1;
    for (int32_t r = 0; r < n; ++r) {
        if (depth[r] >= 0) continue;
        int64_t head = 0, tail = 0;
        depth[r] = 0;
        up[r] = r;
        mx[r] = 0;
        queue[tail++] = r;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int64_t k = start[u]; k < start[u + 1]; ++k) {
                const int64_t e = adj_e[k];
                const int32_t v = adj[k];
                if (!in_msf[e] || depth[v] >= 0) continue;
                depth[v] = depth[u] + 1;
                up[v] = u;
                mx[v] = msf_key(w, e);
                queue[tail++] = v;
            }
        }
    }
    for (int l = 1; l < levels; ++l)
        for (int32_t v = 0; v < n; ++v) {
            const int32_t h = up[(size_t)(l - 1) * n + v];
            up[(size_t)l * n + v] = up[(size_t)(l - 1) * n + h];
            const uint64_t a = mx[(size_t)(l - 1) * n + v], b = mx[(size_t)(l - 1) * n + h];
            mx[(size_t)l * n + v] = a > b ? a : b;
        }
    for (int64_t e = 0; e < m && !rc; ++e) {
        if (in_msf[e]) continue;
        int32_t a = src[e], b = col[e];
        if (a == b) continue;
        uint64_t path = 0;
        if (depth[a] < depth[b]) {
            int32_t t = a;
            a = b;
            b = t;
        }
        for (int l = levels - 1; l >= 0; --l)
            if (depth[a] - (1 << l) >= depth[b]) {
                const uint64_t x = mx[(size_t)l * n + a];
                if (x > path) path = x;
                a = up[(size_t)l * n + a];
            }
        for (int l = levels - 1; l >= 0 && a != b; --l) {
            const int32_t pa = up[(size_t)l * n + a], pb = up[(size_t)l * n + b];
            if (pa != pb) {
                if (mx[(size_t)l * n + a] > path) path = mx[(size_t)l * n + a];
                if (mx[(size_t)l * n + b] > path) path = mx[(size_t)l * n + b];
                a = pa;
                b = pb;
            }
        }
        if (a != b) {
            if (mx[a] > path) path = mx[a];
            if (mx[b] > path) path = mx[b];
            a = up[a];
            b = up[b];
        }
        /* a != b here would mean the ends lie in different trees, which the
         * spanning check has ruled out */
        if (a != b || path > msf_key(w, e)) rc = 3;
    }
done:
    free(src);
    free(uf);
    free(start);
    free(fill);
    free(adj);
    free(adj_e);
    free(queue);
    free(depth);
    free(up);
    free(mx);
    return rc;
}
