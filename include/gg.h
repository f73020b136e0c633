/*
 * gg.h -- C ABI of libgg: single-source shortest paths, breadth-first search
 * and connected components on MI355X (gfx950), hand-written HIP kernels.
 *
 * The problem statement follows the graph DSL paper (Falcon, "Custom Code
 * Generation for a Graph DSL"):
 *   - a graph of points and weighted directed edges is read once (Sec. 2;
 *     Algorithm 1 reads the graph and adds an int point property);
 *   - SSSP lowers t.dist to p.dist + weight(p -> t) with an atomic MIN along
 *     every edge until a sweep changes nothing (Algorithms 1 and 2);
 *   - BFS assigns level lev+1 to every out-neighbour of a level-lev point
 *     whose level is larger, level by level, without atomics (Algorithm 3);
 *   - CC propagates the smallest label over every edge taken both ways until
 *     nothing changes (CC is named in Sec. 4.1; the label convention is this
 *     library's reading: the smallest vertex id of the component);
 *   - each traversal runs vertex-based (CSR: a point and its out-neighbours)
 *     or edge-based (edge list: one work item per edge) (Sec. 3.1, Algorithm
 *     4), and synchronously (topology-driven sweeps ended by a changed flag)
 *     or asynchronously (a data-driven device worklist of updated points,
 *     Sec. 3.3).  The paper picks the variant at compile time; here it is an
 *     argument, and GG_*_AUTO lets the library choose.
 *
 * Values are int32.  INF = GG_INF = 2^31-1 marks an unreached vertex.  The
 * SSSP result is min(shortest distance, INF): a path whose length reaches INF
 * is reported as INF.  Every variant returns bit-identical results.
 *
 * Conventions for every function:
 *   - Return value: GG_OK (0) or a negative gg_status.  Nothing throws.
 *   - Pointers named *_dev are device pointers (hipMalloc'd memory or a torch
 *     tensor's data_ptr); every other pointer is host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Traversal kernels run after the work the caller enqueued earlier on
 *     `stream`.  A traversal takes a data-dependent number of rounds and
 *     only the device can tell when it has ended, so the plain calls
 *     (gg_sssp, gg_bfs, gg_cc and their _ex forms) keep the calling host
 *     thread until the device has reported the end: the output values are
 *     then final, while up to one batch of rounds past the end (which
 *     return at their first instruction) may still be queued on `stream`;
 *     work enqueued on `stream` afterwards runs after them.  The _async
 *     forms (gg_sssp_async and below) return at once with a ticket; one host
 *     thread can so keep several traversals in flight together.
 *   - A HIP failure is reported as GG_EHIP and recorded on the graph handle;
 *     gg_graph_error() returns the first recorded failure.
 */
#ifndef GG_H
#define GG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GG_INF 2147483647

typedef enum {
    GG_OK = 0,
    GG_EINVAL = -1,   /* bad argument: see each function */
    GG_ENOMEM = -2,   /* device or host allocation failed */
    GG_EHIP = -3,     /* a HIP runtime call failed */
    GG_EBUSY = -4,    /* resource in use */
    GG_ENOTSUP = -5,  /* variant not available for this graph */
    GG_ETIMEOUT = -6, /* a traversal exceeded its time limit and stopped */
    GG_EITER = -7     /* a traversal exceeded its iteration bound */
} gg_status;

/* Work distribution (Sec. 3.1): vertex-based over CSR rows, or edge-based
 * with one work item per edge. */
typedef enum { GG_VERTEX = 0, GG_EDGE = 1, GG_MODE_AUTO = 2 } gg_mode;

/* Schedule: synchronous topology-driven sweeps with a changed flag
 * (Algorithms 1-3), or asynchronous data-driven worklist rounds (Sec. 3.3).
 * GG_NEARFAR (SSSP, vertex-based, balanced mapping only) orders the worklist
 * by distance in buckets of width delta -- the Delta-stepping idea the paper
 * credits for the CPU worklist's win on road networks (Sec. 4.2-4.3): a round
 * serves only frontier vertices below the current bound and keeps the rest
 * (with gg_opts.far_degree, only rows longer than it are kept); the bound
 * grows by delta once a round pushes nothing below it.  The result is the
 * same as every other schedule.
 * GG_DIROPT picks the dense or the sparse form of each round on the device,
 * from the size of the frontier the previous round left; it needs the
 * both-directions CSR that GG_SYMMETRIZE or GG_SYMMETRIC provide.
 *   BFS (vertex-based): a small frontier pushes along out-edges as GG_ASYNC
 *   does; a frontier of more than n/12 vertices is pulled -- every unvisited
 *   vertex scans its in-neighbours (the DSL's innbrs iterator, Sec. 2) and
 *   stops at the first one on the level.
 *   CC: round 0 takes one synchronous step from the ids (label = min(id,
 *   smallest neighbour id), read from the both-directions rows without
 *   atomics); later rounds are dense while the rows of the vertices lowered
 *   by the previous round hold more than 1/8 of the both-directions edges,
 *   then serve those vertices as a worklist (GG_ASYNC's vertex form) -- the
 *   paper's synchronous and asynchronous schedules (Sec. 3.3) chosen per
 *   round instead of per run.  A dense round sweeps every stored edge with
 *   atomics (GG_EDGE: GG_SYNC's edge form) or, vertex-based (GG_VERTEX),
 *   lets every vertex pull the labels of its neighbours that are on the
 *   frontier, with no atomics on rows up to the heavy threshold.
 *   SSSP (vertex-based; needs the in-edge CSR of GG_TRANSPOSE): rounds push
 *   the frontier as GG_ASYNC does; a round whose frontier's out-edges exceed
 *   1/4 of the stored edges is pulled instead -- every vertex takes the
 *   least dist[u] + w over its in-edges whose tail u is on the frontier.
 * With GG_MODE_AUTO an explicit GG_DIROPT takes the mode it runs in (edge
 * for CC, vertex otherwise).
 * GG_UNIONFIND (CC only, vertex-based; needs the both-directions CSR): the
 *   components through the DSL's Set type, a union-find structure (Sec. 2):
 *   every vertex is linked with its first and then its second neighbour
 *   (each pass followed by a compression), the root most of 1024 sampled
 *   vertices share is taken as the giant component's, and only the vertices
 *   outside it link their remaining neighbours (Sutton, Ben-Nun and Barak's
 *   Afforest).  Linking hangs the larger root under the smaller, so the
 *   labels are the same: the smallest id of each component.  Four rounds,
 *   whatever the graph's diameter. */
typedef enum {
    GG_SYNC = 0,
    GG_ASYNC = 1,
    GG_SCHED_AUTO = 2,
    GG_NEARFAR = 3,
    GG_DIROPT = 4,
    GG_UNIONFIND = 5
} gg_sched;

/* How vertex-based work is mapped to lanes.  THREAD: one lane walks a whole
 * row (the paper's generated GPU code); WAVE: one wavefront per vertex;
 * BALANCED: a wavefront shares the edges of 64 rows lane by lane, and rows
 * longer than the heavy threshold are cut into fixed chunks spread over the
 * grid.  Ignored for edge-based work. */
typedef enum { GG_MAP_AUTO = 0, GG_MAP_THREAD = 1, GG_MAP_WAVE = 2, GG_MAP_BALANCED = 3 } gg_mapping;

typedef enum { GG_ALGO_SSSP = 0, GG_ALGO_BFS = 1, GG_ALGO_CC = 2, GG_ALGO_MSF = 3 } gg_algo;

/* gg_graph_upload flags */
#define GG_SYMMETRIZE 1u      /* also build the both-directions CSR needed by vertex-based CC */
#define GG_INPUT_ON_DEVICE 2u /* row_ptr/col/w are device pointers */
#define GG_SYMMETRIC 4u       /* the input already holds v->u for every u->v */
#define GG_TRANSPOSE 8u       /* also build the weighted in-edge CSR that the pull rounds of
                                 SSSP's per-round schedule read (8 bytes per edge) */
#define GG_RENUMBER 16u       /* store the graph with its vertices renumbered, hottest first */
#define GG_KEEP_ORDER 32u     /* never renumber */

/* Vertex order in device memory.  The traversals gather the value of an
 * edge's head once per edge, so a vertex is gathered as often as it has
 * in-edges.  On a skewed graph (largest out-degree >= 128 x the mean) of at
 * least 2^20 edges, and on any graph uploaded with GG_RENUMBER, the library
 * stores the graph with its vertices numbered by descending total degree
 * (out + in; ties in the caller's order), so that the values gathered most
 * often share a few cache lines that stay in each die's L2, and each row's
 * edges are stored ordered by head, so that the heads a wavefront gathers
 * at once share lines too.  Nothing of this shows at the interface: every
 * vertex id and edge index passed in or written out is the caller's
 * (sources, dist/level/label outputs -- a CC label is the smallest of the
 * caller's ids in the component -- and the forest flags of gg_msf).  A
 * traversal of a renumbered graph computes into workspace memory and ends
 * with one pass that writes out_dev in the caller's order (CC: a
 * per-component minimum of the caller's ids, then that pass); the
 * workspace holds 8 more bytes per vertex for it, the graph 4 bytes per
 * vertex (both orders) and 8 bytes per edge (the forest's edge map).
 * GG_KEEP_ORDER turns renumbering off; gg_graph_order reports it. */

typedef struct gg_graph_s* gg_graph;
typedef struct gg_ws_s* gg_ws;

/* Per-call options.  Zero-initialise, then set what you need.  Note that a
 * zeroed struct names vertex-based synchronous sweeps (GG_VERTEX and
 * GG_SYNC are 0); GG_MODE_AUTO, GG_SCHED_AUTO and GG_MAP_AUTO ask for the
 * tuned choice, and a NULL opts pointer asks for it in every field. */
typedef struct {
    int32_t mode;          /* gg_mode */
    int32_t sched;         /* gg_sched */
    int32_t mapping;       /* gg_mapping */
    int32_t block_threads; /* 0 = library default (256); else 64..1024, multiple of 64 */
    int32_t max_blocks;    /* 0 = fill the device; else a cap on the persistent grid */
    int32_t heavy_threshold; /* ignored: the rows chunked by the BALANCED mapping are
                                fixed per graph at upload (longer than 16 edges when the
                                largest out-degree is >= 128x the mean, else 32) */
    int32_t time_limit_ms; /* 0 = default (60000); no round is launched after it (GG_ETIMEOUT) */
    int32_t flags;         /* GG_OPT_* bits */
    int32_t delta;         /* GG_NEARFAR bucket width; 0 = default (from the average weight) */
    int32_t hops;          /* local expansion of worklist rounds (GG_ASYNC or GG_NEARFAR,
                              vertex-based, BALANCED mapping), 0..64; 0 = off.  A wavefront
                              serves the vertices it has just lowered (those below the
                              near-far bound) again in the same round, up to `hops` times,
                              from a 128-entry list of its own; what does not fit, and the
                              list left after the last pass, goes to the next round's
                              frontier.  Fewer rounds on high-diameter graphs; the result
                              is the same.  Ignored by other variants; with
                              GG_SCHED_AUTO the tuned choice sets it. */
    int32_t far_degree;    /* GG_NEARFAR: only frontier vertices with more than far_degree
                              out-edges wait for the bound; shorter rows are served at once.
                              0 = every vertex waits (plain near-far).  On skewed graphs the
                              long rows are where a premature expansion costs most, so
                              deferring only them saves most of the repeated work in fewer
                              rounds.  >= 0; with GG_SCHED_AUTO the tuned choice sets it. */
    int32_t reserved[1];
} gg_opts;

/* gg_opts.flags */
#define GG_OPT_CC_NO_JUMP 1u /* CC: plain label propagation, without the label[label[v]]
                                shortcut (the result is the same; the shortcut only
                                shortens high-diameter graphs) */
#define GG_OPT_PROFILE 2u    /* record a HIP event pair around every kernel launch of the
                                call (on the caller's stream); read with gg_last_profile */
/* SSSP with local expansion (hops > 0): how the passes over a wavefront's
 * own list relax.  Checked: a plain load of the head value first, the atomic
 * minimum only when it would lower it.  Direct: the atomic minimum at once
 * (one memory round trip fewer per pass, one atomic more per edge that does
 * not lower its head).  Neither flag: direct on graphs that gg_graph_probe
 * found deep (depth class 2), where rounds are chains of passes run by few
 * wavefronts, checked otherwise.  The result is the same either way. */
#define GG_OPT_LISTS_CHECKED 4u
#define GG_OPT_LISTS_DIRECT 8u

/* Statistics of the last traversal run on a workspace. */
typedef struct {
    int32_t algo, mode, sched, mapping; /* the variant that ran (AUTO resolved) */
    int32_t status;                     /* device-side gg_status of that run */
    int32_t iterations;                 /* sweeps, levels or worklist rounds */
    int32_t grid_blocks, block_threads; /* launch shape */
    int64_t edges_processed;            /* edge relaxations attempted */
    int64_t vertices_processed;         /* vertex visits (rows scanned or worklist entries) */
    int64_t updates;                    /* successful decreases / level writes */
    int64_t pushes;                     /* worklist insertions */
    int64_t reserved[4];
} gg_stats;

/* Per-kernel-kind timing and work of the last traversal run with
 * GG_OPT_PROFILE.  Kinds: 0 = round kernels (sweeps / worklist rounds),
 * 1 = heavy-row chunk kernels, 2 = auxiliary kernels (init, CC shortcut).
 * swept_edges: the part of edges_processed read by the edge sweeps of CC
 * under GG_DIROPT (the rest went through the worklist). */
#define GG_KINDS 3
typedef struct {
    int32_t launches;
    float total_ms;   /* sum of per-launch event times */
    int64_t edges_processed, vertices_processed, updates, pushes;
    int64_t swept_edges;
} gg_kind_profile;

typedef struct {
    int32_t profiled; /* 0 when the last run was not profiled */
    int32_t rounds;   /* round kernels launched (including those past the end) */
    gg_kind_profile kind[GG_KINDS];
    /* device time of the begin of the first launch and of the end of the
     * last, in ms from one reference point per process (an event recorded
     * by the first profiled call), so that traversals run on different
     * streams or host threads can be placed on one time line */
    double begin_ms, end_ms;
} gg_profile;

/* Upload a graph given in CSR: row_ptr[n+1] (row_ptr[0] == 0,
 * non-decreasing, row_ptr[n] == m), col[m] in [0, n), w[m] >= 0 or NULL for
 * an unweighted graph.  Rows need not be sorted.  Host arrays are copied;
 * with GG_INPUT_ON_DEVICE the device arrays are copied on `stream`.  The
 * handle owns every device array it builds: the CSR, the edge list (source
 * of each edge), the static heavy-row chunks, the both-directions CSR when
 * GG_SYMMETRIZE is given, and one default workspace.  Validation runs on the
 * host for host input.  Returns GG_EINVAL for n < 1, m < 0, m >= 2^31, a
 * malformed row_ptr, a column out of range or a negative weight; GG_ENOMEM
 * when device memory runs out.  The call returns when the upload is
 * complete. */
int gg_graph_upload(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                    const int32_t* w, uint32_t flags, void* stream, gg_graph* out);

/* Free a graph and its default workspace.  Workspaces made with
 * gg_ws_create must be freed first, and no host-asynchronous traversal of
 * the graph may be in flight (GG_EBUSY otherwise).  Synchronises the device
 * before freeing. */
int gg_graph_free(gg_graph g);

/* Sizes and degree facts.  Any pointer may be NULL. */
int gg_graph_info(gg_graph g, int32_t* n, int64_t* m, int32_t* max_out_degree,
                  int32_t* has_weights, int32_t* has_sym);

/* First HIP failure recorded on the handle (GG_OK if none). */
int gg_graph_error(gg_graph g);

/* *renumbered = 1 when the graph is stored in the library's own vertex
 * order (see GG_RENUMBER), else 0. */
int gg_graph_order(gg_graph g, int32_t* renumbered);

/* SSSP from `source` (Algorithms 1-2).  dist_out_dev: device int32[n],
 * caller-owned, overwritten.  GG_EINVAL: source outside [0, n), NULL output,
 * or an unweighted graph.  Uses the graph's default workspace. */
int gg_sssp(gg_graph g, int32_t source, int32_t mode, int32_t sched, int32_t* dist_out_dev,
            void* stream);

/* BFS levels from `source` (Algorithm 3).  Same conventions as gg_sssp;
 * weights are ignored. */
int gg_bfs(gg_graph g, int32_t source, int32_t mode, int32_t sched, int32_t* dist_out_dev,
           void* stream);

/* Connected components, label = smallest vertex id of the component, every
 * edge taken both ways.  label_out_dev: device int32[n].  Vertex-based CC
 * needs the both-directions CSR (GG_SYMMETRIZE or GG_SYMMETRIC at upload):
 * GG_ENOTSUP otherwise.  Edge-based CC works on any graph. */
int gg_cc(gg_graph g, int32_t mode, int32_t sched, int32_t* label_out_dev, void* stream);

/* Workspaces: per-query scratch (worklists, stamps, counters) so that
 * several traversals of one graph can be in flight on different streams.
 * A workspace serves one traversal at a time: a call on a workspace that
 * another host thread is using at that moment, or that a host-asynchronous
 * traversal holds, returns GG_EBUSY (the graph's default workspace included),
 * and a call on a workspace whose previous traversal ran on another stream
 * waits for it on the device.  gg_ws_free: GG_EBUSY while a traversal holds
 * the workspace; else waits for its last traversal, then frees it. */
int gg_ws_create(gg_graph g, gg_ws* out);
int gg_ws_free(gg_ws ws);

/* Full-control forms.  ws NULL = the graph's default workspace; opts NULL =
 * all defaults (AUTO everything). */
int gg_sssp_ex(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
               void* stream);
int gg_bfs_ex(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
              void* stream);
int gg_cc_ex(gg_graph g, gg_ws ws, const gg_opts* opts, int32_t* label_out_dev, void* stream);

/* ---- Host-asynchronous traversals: the paper's asynchronous execution
 * (Sec. 3.2, Algorithms 5-6) lets independent kernels -- BFS and SSSP of one
 * graph -- run with no host barrier between them.  These forms validate the
 * call, enqueue the init kernel and the first rounds, hand the traversal to
 * a driver thread of the library and return at once with a ticket.  The
 * rounds run on one of eight streams of the library (taken in turn; the
 * first call makes them), after the work the caller enqueued on `stream`
 * before the call and after the workspace's previous traversal; the driver
 * thread launches the next
 * batch of rounds of every traversal in flight as soon as the previous one
 * completes.  Same arguments, results and errors as the _ex forms, plus:
 *   ticket  (host, out) the handle of the traversal, freed by gg_ticket_free.
 * The workspace (ws NULL = the graph's default one) stays taken until the
 * traversal ends: any call on it meanwhile, gg_last_stats and gg_ws_free
 * included, returns GG_EBUSY, and gg_graph_free returns GG_EBUSY while any
 * traversal of the graph is in flight.  The output must not be read, and
 * the graph not freed, before the ticket reports the end. */
typedef struct gg_ticket_s* gg_ticket;

int gg_sssp_async(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts,
                  int32_t* dist_out_dev, void* stream, gg_ticket* ticket);
int gg_bfs_async(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
                 void* stream, gg_ticket* ticket);
int gg_cc_async(gg_graph g, gg_ws ws, const gg_opts* opts, int32_t* label_out_dev, void* stream,
                gg_ticket* ticket);

/* GG_EBUSY while the traversal runs; once every kernel of it has completed,
 * its status (GG_OK, GG_ETIMEOUT, GG_EITER or a HIP failure).  Never blocks. */
int gg_ticket_query(gg_ticket t);

/* Block the host until every kernel of the traversal has completed; returns
 * its status as gg_ticket_query does. */
int gg_ticket_wait(gg_ticket t);

/* Make `stream` wait on the device for the traversal's last kernel.  The
 * host blocks only until the driver has seen the end (the device work past
 * it is waited for by `stream`, not by the host).  Returns the status. */
int gg_ticket_stream_wait(gg_ticket t, void* stream);

/* Device times of the traversal in milliseconds, measured from the begin of
 * traversal `ref` (NULL = t itself): begin (before its init kernel) and end
 * (after its last round); rounds launched.  Waits for both traversals.  Any
 * output pointer may be NULL. */
int gg_ticket_times(gg_ticket t, gg_ticket ref, float* begin_ms, float* end_ms, int32_t* rounds);

/* Release a ticket (waits for the traversal first if it still runs). */
int gg_ticket_free(gg_ticket t);

/* BFS for callers that cannot allocate memory (code that must not call
 * hipMalloc, such as tight serving loops or hosts that forbid it): the same
 * traversal as gg_bfs_ex on the graph's arrays, with the scratch memory that
 * a workspace holds (frontier flags, heavy-row bits, control and counters,
 * the levels of a renumbered graph in the library's order) taken from one
 * fixed device array of the library, about 27 MB, that each
 * GPU holds from the first call on it until the process ends.  The call
 * allocates nothing: no device or host memory, no events.  Arguments as
 * gg_bfs_ex without a workspace; GG_OPT_PROFILE is ignored and gg_last_stats
 * does not report these calls.  GG_EINVAL for a graph of more than 4,194,304
 * vertices (the array's limit) and for the errors of gg_bfs_ex.  Calls on one
 * GPU share the array: they are serialised by a lock inside the library, and
 * each returns only once every kernel it enqueued on `stream` has completed
 * (the host waits for `stream`), so a call never sees another's kernels. */
int gg_bfs_noalloc(gg_graph g, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
                   void* stream);

/* Minimum spanning forest (MST is the fourth algorithm of Sec. 4.1, Table 3;
 * the DSL's Set type is a union-find structure, Sec. 2).  Every stored edge e
 * is taken as an undirected edge with key (w[e], e) -- weight first, then
 * the edge's index in the uploaded CSR -- so the forest of least keys is
 * unique; self-loops never belong to it.  Boruvka rounds on the device: each
 * component offers its least crossing edge (64-bit atomic minimum), the
 * offered edges join the forest and their components merge in a lock-free
 * union-find.  in_msf_dev: caller-owned device uint8[m], set to 1 for the
 * forest's edges and 0 for the others.  total_weight, n_edges (host,
 * nullable): the forest's summed weight and edge count.  ws NULL = the
 * graph's default workspace (the first call on a workspace allocates 12
 * bytes per vertex for the union-find, kept until the workspace is freed).
 * GG_EINVAL for an unweighted graph or a NULL output with m > 0.  Returns
 * when the forest is complete. */
int gg_msf(gg_graph g, gg_ws ws, uint8_t* in_msf_dev, int64_t* total_weight, int64_t* n_edges,
           void* stream);

/* Statistics of the last traversal on a workspace (NULL = default).  Waits
 * for that traversal to finish.  Returns the traversal's device-side status
 * (GG_ETIMEOUT, GG_EITER) if it failed, GG_OK otherwise; GG_EBUSY while a
 * traversal holds the workspace. */
int gg_last_stats(gg_graph g, gg_ws ws, gg_stats* out);

/* Timing of the last traversal on a workspace (NULL = default) run with
 * GG_OPT_PROFILE.  Waits for the traversal to finish; GG_EBUSY while a
 * traversal holds the workspace. */
int gg_last_profile(gg_graph g, gg_ws ws, gg_profile* out);

/* Resolve AUTO fields of opts for an algorithm on this graph, as a call
 * would (the autotuner's table, else built-in rules). */
int gg_resolve(gg_graph g, int32_t algo, const gg_opts* in, gg_opts* out);

/* ---- Autotuning: the adaptive choice of variant (the paper picks vertex-
 * or edge-based, synchronous or asynchronous processing per input, Sec. 1
 * and Sec. 4.3; here the choice is measured, not fixed at compile time).
 *
 * A graph falls in a class:
 *   size_class  = floor(log2(max(m, 1)) / 2)
 *   skew_class  = 0 if max_out_degree < 8 x average degree, 1 if < 128 x, else 2
 *   depth_class = 0 if a BFS from the highest-degree vertex has < 16 levels,
 *                 1 if < 256, else 2; -1 until gg_graph_probe measured it.
 * A tuning table maps (algo, class) to a variant.  AUTO fields resolve to the
 * entry of the same algorithm with the smallest distance
 *   |size difference| + 4 x [skew differs] + 4 x [depth differs, both known],
 * or to built-in rules when the table has no entry for the algorithm. */
typedef struct {
    int32_t algo, size_class, skew_class, depth_class; /* depth -1 = any */
    int32_t mode, sched, mapping;
    int32_t delta_eighths; /* GG_NEARFAR: bucket width in eighths of the mean edge weight,
                              0..2^23 (0 = 32, four mean weights) */
    int32_t hops;       /* gg_opts.hops of the variant, 0..64; nonzero only for vertex-based
                           GG_ASYNC or GG_NEARFAR with the BALANCED (or AUTO) mapping */
    int32_t far_degree; /* gg_opts.far_degree of the variant, >= 0; nonzero only for
                           GG_NEARFAR */
} gg_tune_entry;

/* Replace the process-wide tuning table (count 0 clears it).  The entries
 * are copied.  GG_EINVAL for a NULL table with count > 0, a negative count or
 * an entry with an out-of-range field. */
int gg_tune_set(const gg_tune_entry* entries, int32_t count);

/* Number of entries in the table; copies up to `cap` of them to `out`. */
int gg_tune_get(gg_tune_entry* out, int32_t cap);

/* Class of a graph of these sizes (pure host computation; levels < 0 =
 * unknown depth). */
int gg_class_of(int64_t m, int32_t n, int32_t max_out_degree, int32_t levels,
                int32_t* size_class, int32_t* skew_class, int32_t* depth_class);

/* Variant the table (else the built-in rules) picks for an algorithm and a
 * class, as gg_resolve would: `out` receives the query's algorithm and class
 * and the chosen variant fields (mapping AUTO reported as BALANCED). */
int gg_tune_lookup(int32_t algo, int32_t size_class, int32_t skew_class, int32_t depth_class,
                   gg_tune_entry* out);

/* Measure the graph's depth class (one BFS on `stream`, waited for) and keep
 * it on the handle; later AUTO resolutions use it. */
int gg_graph_probe(gg_graph g, void* stream);

/* Class of an uploaded graph (depth -1 until probed). */
int gg_graph_class(gg_graph g, int32_t* size_class, int32_t* skew_class, int32_t* depth_class);

/* ---- Batched traversals: many independent SSSP/BFS instances of uneven
 * size in one launch sequence.  The paper observed that one traversal kernel
 * already used all GPU resources on its hardware (Sec. 4.4); small instances
 * do not, so here they are packed together.  Instances of the same algorithm
 * and graph class (gg_class_of) are concatenated into one graph with
 * per-instance vertex offsets, so every instance is a separate component
 * and one multi-source traversal of the group computes all of them exactly
 * as separate calls would (bit-identical).  Each group runs in the variant
 * the tuner picks for the group's graph (a near-far pick runs as the plain
 * worklist: the buckets pay off on large single-source traversals, not on a
 * group of small ones), on a stream of its own; after the
 * first run the group's launch sequence is captured in a HIP graph and later
 * runs replay it (rounds past the end return at once; a replay that stops
 * short is continued with eager launches).  Not thread-safe per batch. */
typedef struct gg_batch_s* gg_batch;

typedef struct {
    int32_t algo;            /* GG_ALGO_SSSP or GG_ALGO_BFS */
    int32_t n;               /* vertices (>= 1) */
    int64_t m;               /* edges */
    const int32_t* row_ptr;  /* host CSR, same rules as gg_graph_upload */
    const int32_t* col;
    const int32_t* w;        /* weights (SSSP: required; BFS: ignored, may be NULL) */
    int32_t source;          /* in [0, n) */
    int32_t reserved;
} gg_instance;

#define GG_BATCH_NO_GRAPH 1u  /* enqueue eagerly on every run (no HIP graph capture) */
#define GG_BATCH_ONE_GROUP 2u /* one group per algorithm, no split by class */

/* Build a batch from host instances (copied).  GG_EINVAL for count < 1 or an
 * invalid instance (bad algorithm, source out of range, malformed CSR,
 * negative weight, SSSP without weights, more than 2^31 - 1 vertices or
 * edges in one group).  The call returns when the upload is complete. */
int gg_batch_create(const gg_instance* inst, int32_t count, uint32_t flags, void* stream,
                    gg_batch* out);

/* Run every instance.  out_dev: device int32 array of gg_batch_info's
 * total_n entries; instance i's result is out_dev[v_off[i] .. v_off[i]+n_i)
 * with v_off from gg_batch_offsets.  Enqueued on `stream` (the groups run on
 * streams of their own that wait for and are waited by `stream`); the call
 * returns once every group has finished its rounds. */
int gg_batch_run(gg_batch b, int32_t* out_dev, void* stream);

/* v_off[i] for each instance (count entries). */
int gg_batch_offsets(gg_batch b, int64_t* v_off);

/* Totals: groups, vertices (the length of out_dev), edges. */
int gg_batch_info(gg_batch b, int32_t* groups, int64_t* total_n, int64_t* total_m);

/* Group g: algorithm, instances, vertices, edges, the variant it runs, the
 * rounds captured in its HIP graph (0 = not captured) and its last round
 * count.  Outputs may be NULL. */
int gg_batch_group(gg_batch b, int32_t g, int32_t* algo, int32_t* instances, int64_t* n,
                   int64_t* m, int32_t* mode, int32_t* sched, int32_t* mapping,
                   int32_t* captured_rounds, int32_t* last_rounds);

/* Free a batch (waits for its work). */
int gg_batch_free(gg_batch b);

/* ---- Serving: SSSP/BFS queries admitted as they arrive (continuous
 * batching).  A server holds resident graphs (added after gg_graph_upload;
 * the server owns them from then on), a FIFO of submitted queries and a set
 * of slots.  A driver thread of the server admits queued queries while a
 * slot is free and the per-query state of all admitted queries (a
 * workspace: frontier flags and heavy-row bits, ~2.3 bytes per vertex) fits the
 * memory budget, enqueues each admitted query's rounds on the slot's own
 * stream, and launches a query's next batch of rounds as soon as its
 * previous one completes, so the kernels of different queries overlap on
 * the device.  A query's result is bit-identical to the same call made
 * alone.  Every call may come from any thread. */
typedef struct gg_server_s* gg_server;

typedef struct {
    int64_t id;           /* from gg_server_submit */
    int32_t status;       /* GG_OK or the traversal's error */
    int32_t rounds;       /* rounds the traversal took */
    double t_submit, t_admit, t_done; /* seconds on the server's steady clock */
} gg_query_result;

/* slots: queries in flight at most (1..1024); mem_budget_bytes: bound on the
 * per-query state of queries in flight (0 = no bound). */
int gg_server_create(int32_t slots, int64_t mem_budget_bytes, gg_server* out);

/* Hand a graph to the server; *graph_id names it in submissions. */
int gg_server_add_graph(gg_server s, gg_graph g, int32_t* graph_id);

/* Retire a graph: later submissions to it fail; queries already queued or
 * in flight finish.  Its memory (graph and pooled workspaces) is released
 * by the driver thread once none of its queries is left and the server has
 * no query in flight (releasing device memory waits for the whole device),
 * or by gg_server_free. */
int gg_server_remove_graph(gg_server s, int32_t graph_id);

/* Queue a query.  out_dev: caller-owned device int32[n] of that graph,
 * written by the traversal (readable once the query is reported done; the
 * caller keeps it allocated until then).  stream: the query's kernels run
 * after the work enqueued on it before this call (an event recorded there),
 * so the caller may prepare out_dev on its stream.  GG_EINVAL for an
 * unknown or retiring graph, a bad algorithm or source.  With a memory
 * budget, the workspaces kept for reuse count against it too: idle ones of
 * other graphs are freed when a new one would not fit. */
int gg_server_submit(gg_server s, int32_t graph_id, int32_t algo, int32_t source,
                     int32_t* out_dev, void* stream, int64_t* query_id);

/* Copies up to `cap` newly finished queries to results and their count to
 * *n_done.  Never blocks on the device. */
int gg_server_poll(gg_server s, gg_query_result* results, int32_t cap, int32_t* n_done);

/* Queued, in-flight and retained-state counts, memory of in-flight state. */
int gg_server_state(gg_server s, int32_t* queued, int32_t* in_flight, int64_t* state_bytes);

/* Seconds on the server's clock (the clock of gg_query_result). */
double gg_server_now(gg_server s);

/* Stop the driver thread (queries still queued are dropped), wait for the
 * device work already enqueued, free the graphs the server owns and the
 * server. */
int gg_server_free(gg_server s);

/* Human-readable status name. */
const char* gg_status_str(int32_t status);

/* Library version, for the binding's compatibility check. */
int32_t gg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GG_H */
