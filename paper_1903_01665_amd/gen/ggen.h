/*
 * ggen.h -- seeded synthetic graph generators (host C, no GPU).
 *
 * This module only synthesises inputs.  It holds none of the traversal
 * arithmetic: it draws random numbers, builds edge lists and sorts them into
 * CSR.  Both the GPU path and the CPU oracle consume its output, so it lives
 * in a module of its own.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) seeds xoshiro256**
 * (Blackman & Vigna, "Scrambled linear pseudorandom number generators",
 * 2018).  Every (seed, stream, chunk) triple owns an independent generator,
 * so output does not depend on the number of host threads used.
 *
 * Graph format produced: CSR with rows sorted by source vertex, edges of a
 * row kept in generation order (stable counting sort).  row_ptr[n+1], col[m],
 * w[m], all int32; m must stay below 2^31.
 *
 * Integer draw in [lo, hi]: lo + ((r >> 32) * (hi - lo + 1) >> 32), using the
 * top 32 bits of one xoshiro256** output (multiply-shift, no rejection).
 *
 * All functions return 0 on success and a negative value on bad arguments.
 * Output buffers are caller-owned host memory of the stated sizes.
 */
#ifndef GGEN_H
#define GGEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One raw xoshiro256** output stream, seeded from (seed, stream, chunk).
 * Writes count 64-bit outputs to out.  Exposed for generator tests. */
int ggen_raw(uint64_t seed, uint64_t stream, uint64_t chunk, int64_t count, uint64_t* out);

/* Uniform directed random graph: m edges, both endpoints uniform in [0, n),
 * self-loops rejected and redrawn (so exactly m edges), duplicates kept,
 * weights uniform in [wlo, whi].  w may be NULL (no weights drawn). */
int ggen_uniform(int32_t n, int64_t m, int32_t wlo, int32_t whi, uint64_t seed, uint64_t stream,
                 int32_t* row_ptr, int32_t* col, int32_t* w);

/* Recursive R-MAT: 2^scale vertices, m edges.  For each edge and each of
 * `scale` levels, u = 53 random bits / 2^53 picks a quadrant by the
 * cumulative bounds (a, a+b, a+b+c): the source bit is set for quadrants c
 * and d, the destination bit for b and d, most significant bit first.  No
 * noise, no vertex permutation, duplicates and self-loops kept.  The weight
 * is drawn after the endpoints from the same stream. */
int ggen_rmat(int32_t scale, int64_t m, double a, double b, double c, int32_t wlo, int32_t whi,
              uint64_t seed, uint64_t stream, int32_t* row_ptr, int32_t* col, int32_t* w);

/* Number of directed edges ggen_grid produces. */
int64_t ggen_grid_edges(int32_t width, int32_t height, int64_t n_shortcuts);

/* Road-like grid: width x height vertices, id = y*width + x.  Every
 * 4-neighbour pair is one undirected edge with one weight draw, stored in
 * both directions.  Then n_shortcuts undirected shortcut edges: u uniform,
 * (dx, dy) uniform in [-span, span]^2 with |dx|+|dy| >= 2 (never a grid
 * edge), offsets redrawn until the target is on the grid; one weight draw,
 * both directions stored. */
int ggen_grid(int32_t width, int32_t height, int64_t n_shortcuts, int32_t span, int32_t wlo,
              int32_t whi, uint64_t seed, uint64_t stream, int32_t* row_ptr, int32_t* col,
              int32_t* w);

/* Stable CSR build from an edge list (exposed so tests can hand-build
 * graphs).  Rows sorted by src, generation order kept inside a row. */
int ggen_csr_from_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* wt, int32_t* row_ptr, int32_t* col, int32_t* w);

/* `count` sources drawn uniformly among vertices with out-degree > 0
 * (rejection sampling).  Returns -2 when no vertex has an out-edge. */
int ggen_pick_sources(int32_t n, const int32_t* row_ptr, int32_t count, uint64_t seed,
                      uint64_t stream, int32_t* out);

/* FNV-1a 64 hash over the bytes of an int32 array (regression checks). */
uint64_t ggen_fnv1a(const int32_t* a, int64_t count);

#ifdef __cplusplus
}
#endif
#endif
