/*
 * oracle.h -- CPU reference results for SSSP, BFS and connected components.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, helper or table with the GPU library; the two meet only through
 * the plain CSR arrays the input generator produces.
 *
 * Every function is a plain, sequential, obviously-correct CPU routine
 * (and MSF, the minimum spanning forest, as below):
 *   - the paper's fixpoint methods (vertex/edge relaxation sweeps with an
 *     atomic MIN and a changed flag, Algorithms 1-2; level-synchronous BFS,
 *     Algorithm 3; CC by label propagation, named in Sec. 4.1) reach exactly
 *     the plain definitions below, so the oracle computes those definitions:
 *       SSSP  dist[v] = min over directed paths s->v of the summed weights,
 *             clamped to INF = 2^31-1 (INF also means "no path");
 *       BFS   dist[v] = number of edges on a shortest directed path s->v,
 *             INF when none;
 *       CC    label[v] = smallest vertex id in v's component of the graph
 *             with every edge taken in both directions.
 *   - brute-force routines (Floyd-Warshall, Bellman-Ford, Warshall closure)
 *     for tiny graphs, used to pin the main routines;
 *   - O(n+m) certificates that accept exactly the correct outputs.
 *
 * Graph arguments: CSR with row_ptr[n+1] (non-decreasing, row_ptr[0] == 0),
 * col[m], w[m] (m = row_ptr[n]), all int32, host memory, read only.
 * Outputs: caller-owned int32 arrays of length n.
 * Return: 0 on success; -1 on invalid arguments (n < 1, source out of range,
 * malformed CSR, column out of range, negative weight, size limit exceeded);
 * -3 when host memory runs out.  The certificate functions return 0 when the
 * output is correct and a positive code naming the violated property.
 */
#ifndef GG_ORACLE_H
#define GG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_INF 2147483647

/* Dijkstra with a binary min-heap (lazy deletion), 64-bit distances. */
int oracle_sssp(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                int32_t source, int32_t* dist);

/* Breadth-first search with a FIFO queue. */
int oracle_bfs(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t source,
               int32_t* dist);

/* Union-find (union by size, path halving) over every edge taken as
 * undirected; label = smallest member id of the set. */
int oracle_cc(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* label);

/* Minimum spanning forest (Kruskal; Sec. 4.1 names MST, Sec. 2 the
 * union-find Set).  Every stored edge e is an undirected edge with key
 * (w[e], e) -- distinct keys, so the forest is unique; self-loops are never
 * in it.  in_msf: caller-owned uint8[m], 1 for the edges of the forest;
 * *total_weight (nullable): their summed weight. */
int oracle_msf(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
               uint8_t* in_msf, int64_t* total_weight);

/* Brute force for tiny graphs (n <= 512). */
int oracle_sssp_floyd_warshall(int32_t n, const int32_t* row_ptr, const int32_t* col,
                               const int32_t* w, int32_t source, int32_t* dist);
int oracle_sssp_bellman_ford(int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* w, int32_t source, int32_t* dist);
int oracle_cc_warshall(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* label);
/* Least-key spanning forest over all edge subsets (n <= 10, m <= 20, w < 2^24). */
int oracle_msf_brute(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                     uint8_t* in_msf);

/* Certificates.
 * SSSP (w == NULL checks BFS levels, every weight taken as 1):
 *   1 dist[source] != 0;  2 a value outside [0, INF];
 *   3 an edge u->v with dist[u] < INF and dist[u] + w < dist[v] (infeasible);
 *   4 the vertices reached from the source along tight edges
 *     (dist[u] + w == dist[v]) are not exactly the vertices with dist < INF.
 * CC:
 *   1 a value outside [0, v];  2 label[label[v]] != label[v];
 *   3 an edge whose endpoints carry different labels;
 *   4 the number of distinct labels differs from the number of components
 *     counted by a breadth-first search over the undirected adjacency. */
int oracle_check_sssp(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                      int32_t source, const int32_t* dist);
int oracle_check_cc(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* label);
/* MSF: 1 the selected edges hold a self-loop or a cycle; 2 they do not span
 * (their count differs from n minus the number of components); 3 an edge
 * left out closes a cycle holding a larger key (cycle property). */
int oracle_check_msf(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                     const uint8_t* in_msf);

#ifdef __cplusplus
}
#endif
#endif
