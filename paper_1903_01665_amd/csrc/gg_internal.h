// gg_internal.h -- structures shared by the kernels and the host runtime of
// libgg.  Not part of the public ABI (include/gg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gg {

constexpr int kInf = 2147483647;
constexpr int kWave = 64;
constexpr int kTile = 64;            // vertices per frontier tile (one wavefront)
constexpr int kMaxStatBlocks = 4096; // per-block statistics slots
// rows longer than the graph's heavy threshold are chunked (balanced
// mapping): 16 on graphs whose largest out-degree is at least 128 times the
// mean, 32 on the others (measured on MI355X: a lower threshold moves more
// edges of a skewed graph into full-wavefront chunks, while on a uniform
// graph it cuts short rows into underfilled chunks)
constexpr int kHeavySkewed = 16;
constexpr int kHeavyUniform = 32;
constexpr int kChunk = 512;          // edges per heavy-row chunk
constexpr int kKinds = 3;            // statistics kinds: round, heavy chunks, auxiliary
constexpr int kParts = 8;            // frontier work items per 64-tile group (8 tiles each)
constexpr int kXcd = 8;              // accelerator dies; workgroups go to them round-robin
enum Kind { KIND_ROUND = 0, KIND_HEAVY = 1, KIND_AUX = 2 };

enum Algo { SSSP = 0, BFS = 1, CC = 2 };
enum Map { MAP_THREAD = 1, MAP_WAVE = 2, MAP_BALANCED = 3 };

// Loop-control block, one per workspace.  Kernels of one traversal read the
// slots written by earlier kernels of the same stream (kernel boundaries make
// them visible); slot r % 3 belongs to round r.
struct Ctl {
    int done;        // set by the first round kernel that finds nothing left to do
    int iters;       // rounds that ran, set together with done
    int changed[4];  // [r % 3]: round r updated or pushed something
    int bound[4];    // near-far schedule: [r % 3] = distance bound of round r
    int near_[4];    // near-far schedule: [r % 3] = round r pushed below its bound
    int grid[4];     // [r % 3] = grid of round r's round kernel (push counts below)
    int hgrid[4];    // [r % 3] = grid of round r's heavy kernel
    int pull[4];     // [r % 3] = round r took the dense form (BFS pull, CC edge sweep)
    int giant;       // CC by union-find: the root most sampled vertices have
    int pad[1];
};

// Per-block counters, summed on the host after a traversal; one array of
// kMaxStatBlocks slots per kernel kind.
struct Stat {
    long long edges, verts, updates, pushes;
    long long swept;  // edges read by the sweeps of a per-round CC schedule
};

// Device view of an uploaded graph.  Arrays are owned by the host-side
// handle.  The CSR keeps the input's row order; src is the edge-list form.
struct DevGraph {
    int n, m;
    const int* row;  // [n+1]
    const int* col;  // [m]
    const int* w;    // [m] or null
    const int* src;  // [m] source vertex of each edge
    // both-directions graph for CC (aliases row/col/src when the input is symmetric)
    int ms;
    const int* srow;
    const int* scol;
    const int* ssrc;
    // heavy rows (degree > heavy) as (row, first edge) chunks of `chunk` edges
    int heavy, chunk;
    const int2* hchunks;
    int n_hchunks;
    const int2* shchunks;
    int n_shchunks;
    bool symmetric;  // input already holds both directions of every edge
    // the edge list again, cut into kXcd parts by head vertex (equal edge
    // counts), each padded to a multiple of 4 with self-loops on vertex 0;
    // null when not built
    const int* psrc;
    const int* pcol;
    const int* pw;
    int poff[kXcd + 1];
    // in-edges with their weights (pull rounds of SSSP): row v of trow/tcol
    // lists the tails of v's in-edges, tw their weights; rows longer than
    // `heavy` are also cut into (row, first edge) chunks; null when not built
    const int* trow;
    const int* tcol;
    const int* tw;
    const int2* tchunks;
    int n_tchunks;
};

// Device view of a workspace: frontier flags (one byte per vertex, one per
// 64-vertex tile), two generations; the heavy frontier rows of a round as a
// bit per vertex, two generations; control; stats.
struct DevWs {
    unsigned char* vflag[2];
    unsigned char* tflag[2];
    unsigned* hbits[2];  // [(n + 31) / 32] each: round r marks its heavy rows in hbits[r & 1]
    Ctl* ctl;
    Stat* stat;
    int* pcount;  // [3][2][kMaxStatBlocks]: frontier size pushed per block of round r % 3
                  // (round, heavy): vertices, or with Round::fedges their row lengths
};

// Everything a round kernel needs.  Passed by value.
struct Round {
    DevGraph g;
    DevWs ws;
    int* val;    // dist or label, [n]
    int source;          // single source (when nsrc == 0)
    const int* sources;  // device list of sources of a multi-source traversal
    int nsrc;
    int r;       // round (sweep, level) index
    int epoch;   // tag of this traversal: grows across the traversals of a workspace
    int* host_done; // pinned host word: set to `epoch` by the kernel that finds the end
    int mapping; // Map
    int jump;    // CC: apply the label[label[v]] shortcut
    int delta;   // SSSP near-far schedule: bucket width (0 = plain worklist rounds)
    int fedges;  // CC per-round dense/sparse choice: push counts are the row lengths
                 // (both-directions CSR) of the pushed vertices, and edge sweeps push
    int hops;    // worklist rounds (balanced mapping): passes of local expansion (0 = off)
    int far_degree; // near-far: only rows longer than this wait for the bound (0 = all)
    int pullmode;   // per-round schedule: dense rounds pull over in-edges (SSSP: trow;
                    // CC: the both-directions rows) instead of pushing or sweeping
    int direct_lists; // SSSP local expansion: list passes issue their atomics without a
                      // check load of the head value
    int* rmin;      // CC on a renumbered graph: per-label minimum of the caller's ids,
                    // filled with INT_MAX by the init kernel (null otherwise)
};

// Launch entry points (gg_kernels.hip).  Each returns the hipError_t of the
// launch.
hipError_t launch_init(const Round& R, int algo, bool async, int grid, int block, hipStream_t s);
hipError_t launch_seed(const Round& R, bool async, int grid, int block, hipStream_t s);
hipError_t launch_vsync(const Round& R, int algo, int grid, int block, hipStream_t s);
hipError_t launch_esync(const Round& R, int algo, int grid, int block, hipStream_t s);
hipError_t launch_vasync(const Round& R, int algo, int grid, int block, hipStream_t s);
hipError_t launch_easync(const Round& R, int algo, int grid, int block, hipStream_t s);
hipError_t launch_heavy(const Round& R, int algo, int grid, int block, hipStream_t s);
hipError_t launch_bfs_diropt(const Round& R, int grid, int block, hipStream_t s);
hipError_t launch_jump(const Round& R, int grid, int block, hipStream_t s);
hipError_t launch_cc_diropt(const Round& R, int grid, int block, hipStream_t s);
hipError_t launch_sssp_diropt(const Round& R, int grid, int block, hipStream_t s);
// CC by union-find (GG_UNIONFIND), phase R.r: link, find the giant root,
// link the rest; and the compression pass after a linking phase
hipError_t launch_uf(const Round& R, int grid, int block, hipStream_t s);
hipError_t launch_uf_compress(const Round& R, int grid, int block, hipStream_t s);
// One thread stores v into the pinned host word *p (system scope) once every
// earlier kernel of the stream has completed.
hipError_t launch_mark(unsigned long long* p, unsigned long long v, hipStream_t s);

// Graph build helpers (gg_kernels.hip).
hipError_t launch_fill_src(const int* row, int n, int m, int* src, int grid, int block,
                           hipStream_t s);
hipError_t launch_count_in(const int* col, int m, int* indeg, int grid, int block, hipStream_t s);
hipError_t launch_sym_fill(const int* row, const int* col, const int* src, int n, int m,
                           const int* srow, int* cursor, int* scol, int grid, int block,
                           hipStream_t s);
hipError_t launch_t_fill(const int* col, const int* w, const int* src, int m, const int* trow,
                         int* cursor, int* tcol, int* tw, int grid, int block, hipStream_t s);
// stats[0..3] = min column, max column, min weight, max weight (initialised
// by the caller to the neutral values); *wsum += the weight sum
hipError_t launch_check(const int* col, const int* w, int m, int* stats,
                        unsigned long long* wsum, int grid, hipStream_t s);
// stable split of the edge list by head part: per-block counts
// (split_blocks(m) x kXcd), then placement from per-block bases
int split_blocks(long long m);
hipError_t launch_split_count(const int* col, int m, const unsigned char* part, int* counts,
                              hipStream_t s);
hipError_t launch_split_place(const int* src, const int* col, const int* w, int m,
                              const unsigned char* part, const long long* base, int* psrc,
                              int* pcol, int* pw, hipStream_t s);
// Renumbering: caller edge e of row u = src[e] goes to place
// nrow[newid[u]] + (e - row[u]) with head newid[col[e]] and weight w[e];
// eorig[place] = e and epos[e] = place.  w and nw may be null.
hipError_t launch_renumber(const int* row, const int* col, const int* w, const int* src, int m,
                           const int* newid, const int* nrow, int* ncol, int* nw, int* eorig,
                           int* epos, int grid, int block, hipStream_t s);
// out[v] = val[newid[v]] for every caller id v; a vertex whose new id is
// >= n_active (no edge) gets 0 if it is the source, else INF
hipError_t launch_unrenumber(int* out, const int* val, const int* newid, int n, int n_active,
                             int source, int grid, int block, hipStream_t s);
// CC: rmin[label[v']] = least oldid[v'] over the vertices v' of each label
hipError_t launch_cc_min_ids(const int* label, const int* oldid, int* rmin, int n, int grid,
                             int block, hipStream_t s);
// CC: out[v] = rmin[label[newid[v]]] for every caller id v (v itself when
// its new id is >= n_active: no edge, a component of its own)
hipError_t launch_cc_min_out(int* out, const int* label, const int* newid, const int* rmin,
                             int n, int n_active, int grid, int block, hipStream_t s);

}  // namespace gg
