// gg_kernels.hip -- traversal kernels of libgg for gfx950 (CDNA4, 64-wide
// wavefronts).
//
// One kernel launch is one round: a synchronous sweep (Algorithms 1-3: every
// vertex or every edge, ended by a changed flag) or one asynchronous worklist
// round (Sec. 3.3: only the vertices updated in the previous round).  The
// host enqueues rounds back to back; every round kernel first reads the
// control block and returns at once when an earlier round found nothing to
// do, so no kernel ever waits on another and every launch terminates.
//
// Relaxation (Algorithms 1-2): for an edge p -> t, t.dist is lowered to
// p.dist + weight with an atomic minimum.  A plain load of t.dist comes
// first and the atomic is skipped when it cannot lower the value; values only
// decrease, so a stale load can only cause an unnecessary atomic, never a
// missed one.
//
// BFS (Algorithm 3): level lev visits the vertices with dist == lev and
// writes lev+1 into every out-neighbour whose level is larger, with plain
// stores (all writers of a level store the same value).
//
// CC: label[t] is lowered to label[p] over every edge, both directions.  The
// optional shortcut label[p] = label[label[p]] keeps label[p] a member of p's
// component, so the fixpoint (the smallest id of the component) is unchanged.
//
// Frontier (asynchronous schedule): one byte per vertex and one per 64-vertex
// tile, two generations.  A push is a plain byte store of 1, so duplicates
// collapse without atomics; a round clears the flags it consumes.  Rows longer
// than the heavy threshold are cut into fixed chunks and placed on a queue
// that a second kernel of the same round spreads over the whole grid.

#include "gg_internal.h"

namespace gg {

// A frontier work item is one kParts-th of a 64-tile group: the wavefront
// checks the tile flags of its part (64 / kParts tiles) and serves the
// flagged ones.  Fewer, larger items make the scan of a sparse frontier
// cheaper (deep graphs run thousands of rounds with small frontiers) at the
// price of balance on dense ones; 8 tiles per item measured best.

// Edges each lane keeps in flight in the relaxation loops.
constexpr int kBatch = 4;

// Edges per lane in flight in the worklist kernels, by algorithm (measured on
// MI355X): BFS stores levels without atomics and gains from more wavefronts
// at once (2); SSSP and CC use 4; the near-far SSSP rounds, whose frontiers
// are small and latency-bound, 8.
constexpr int batch_for(int A, bool nf) { return nf ? 8 : A == BFS ? 2 : 4; }

// Direction-optimizing BFS pulls a level when its frontier holds more than
// n / kPullRatio vertices.  Not 20: er23's level 6 holds 464K of 8.4M
// vertices, and pulling it (most of the unvisited vertices scan their whole
// in-lists in vain) took BFS from 1.06 to 2.0 ms.  16 rather than 12: on
// the renumbered rmat22 the step gains 1.7% (a sweep over 8, 12, 16).
constexpr int kPullRatio = 16;

// CC with the per-round choice sweeps every edge while the rows of the
// frontier hold more than (both-directions edges) / kSweepRatio edges.
constexpr int kSweepRatio = 8;

// SSSP with the per-round choice pulls a round when the out-edges of the
// frontier the previous round left exceed (stored edges) / kSsspPullRatio.
constexpr int kSsspPullRatio = 4;

// ------------------------------------------------------------ helpers ----

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Counters of one lane for the current kernel.
struct Acc {
    int e = 0, v = 0, u = 0, p = 0;
    int nr = 0;  // near-far: pushed a distance below the round's bound
    int f = 0;   // row lengths of the pushed vertices (Round::fedges), saturating
    int d = 0;   // edges read by a sweep of the per-round CC schedule
    __device__ void add_f(int d) { f = f > (1 << 30) - d ? 1 << 30 : f + d; }
};

// Frontier size of round r-1 as its kernels recorded it: the sum of the
// per-block push counts of its round and heavy kernels.  Every block reads
// the same slots, so the result is the same grid-wide.
__device__ long long prev_front(const Round& R) {
    const Ctl* ctl = R.ws.ctl;
    const int slot = (R.r - 1) % 3;
    const int gr = *(volatile const int*)&ctl->grid[slot];
    const int gh = *(volatile const int*)&ctl->hgrid[slot];
    __shared__ long long s_sum[4];
    long long part = 0;
    for (int b = threadIdx.x; b < gr; b += blockDim.x)
        part += R.ws.pcount[(slot * 2 + KIND_ROUND) * kMaxStatBlocks + b];
    for (int b = threadIdx.x; b < gh; b += blockDim.x)
        part += R.ws.pcount[(slot * 2 + KIND_HEAVY) * kMaxStatBlocks + b];
    for (int d = 32; d > 0; d >>= 1) part += __shfl_xor(part, d, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = part;
    __syncthreads();
    long long front = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) front += s_sum[i];
    __syncthreads();
    return front;
}

// Round entry, uniform over the whole grid.  Returns false when the
// traversal has finished: either an earlier round set `done`, or round r-1
// changed nothing, in which case this kernel records the round count.
// The kernel that finds the end also tells the host, by storing this
// traversal's epoch into a pinned host word (older traversals store older
// epochs, so a late kernel of an earlier traversal cannot end this one).
__device__ __forceinline__ bool round_begin(const Round& R) {
    Ctl* ctl = R.ws.ctl;
    if (*(volatile int*)&ctl->done) return false;
    if (R.r > 0 && *(volatile int*)&ctl->changed[(R.r - 1) % 3] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->iters = R.r;
            ctl->done = 1;
            __hip_atomic_store(R.host_done, R.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return false;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // slots of round r+1: last read by rounds that have completed
        ctl->changed[(R.r + 1) % 3] = 0;
    }
    return true;
}

// Near-far schedule (SSSP, delta > 0): round r serves only the frontier
// vertices whose distance is below the bound B_r and keeps the others on the
// frontier (with Round::far_degree > 0 only the rows longer than it are
// kept; shorter ones are served whatever their distance).  B_0 = delta;
// B_r = B_{r-1} while round r-1 pushed some distance below B_{r-1}, else
// B_{r-1} + delta.  Every block derives B_r from the slots of round r-1, so
// the choice is the same grid-wide; block 0 records it.
__device__ __forceinline__ int nearfar_bound(const Round& R) {
    Ctl* ctl = R.ws.ctl;
    int b = R.delta;
    if (R.r > 0) {
        const int pb = *(volatile int*)&ctl->bound[(R.r - 1) % 3];
        const bool near = *(volatile int*)&ctl->near_[(R.r - 1) % 3] != 0;
        b = near ? pb : (pb > kInf - R.delta ? kInf : pb + R.delta);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->bound[R.r % 3] = b;
        ctl->near_[(R.r + 1) % 3] = 0;
    }
    return b;
}

__device__ __forceinline__ void nearfar_finish(const Round& R, const Acc& acc) {
    if (__syncthreads_or(acc.nr) && threadIdx.x == 0) R.ws.ctl->near_[R.r % 3] = 1;
}

// Block-level reduction of the lane counters; one plain update of this
// block's statistics slot (row `kind`) and, when anything changed, of the
// round's flag.  The block's frontier count goes to push-count row `pk`: the
// kind's own row by default, none for the auxiliary kind.
__device__ void block_finish(const Round& R, const Acc& a, int slot, int kind, int pk = -1) {
    __shared__ long long s_acc[4][6];
    int e = wave_sum(a.e), v = wave_sum(a.v), u = wave_sum(a.u), p = wave_sum(a.p);
    int dd = wave_sum(a.d);
    long long f = a.f;
    for (int d = 32; d > 0; d >>= 1) f += __shfl_xor(f, d, 64);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_acc[wid][0] = e;
        s_acc[wid][1] = v;
        s_acc[wid][2] = u;
        s_acc[wid][3] = p;
        s_acc[wid][4] = f;
        s_acc[wid][5] = dd;
    }
    __syncthreads();
    if (pk < 0 && kind != KIND_AUX) pk = kind;
    if (threadIdx.x == 0) {
        long long E = 0, V = 0, U = 0, P = 0, F = 0, D = 0;
        for (int i = 0; i < nw; ++i) {
            E += s_acc[i][0];
            V += s_acc[i][1];
            U += s_acc[i][2];
            P += s_acc[i][3];
            F += s_acc[i][4];
            D += s_acc[i][5];
        }
        if (E | V | U | P) {
            Stat* st = R.ws.stat + kind * kMaxStatBlocks + blockIdx.x;
            st->edges += E;
            st->verts += V;
            st->updates += U;
            st->pushes += P;
            st->swept += D;
        }
        if (U > 0 || P > 0) R.ws.ctl->changed[slot] = 1;
        // frontier pushed by this block in this round (every block writes its
        // slot): vertices, or their row lengths
        if (pk >= 0) {
            const long long c = R.fedges ? F : P;
            R.ws.pcount[(slot * 2 + pk) * kMaxStatBlocks + blockIdx.x] =
                (int)(c < 2147483647LL ? c : 2147483647LL);
        }
        if (blockIdx.x == 0) {
            if (pk == KIND_ROUND) R.ws.ctl->grid[slot] = gridDim.x;
            if (pk == KIND_HEAVY) R.ws.ctl->hgrid[slot] = gridDim.x;
        }
    }
}

// Lanes hold one row each, [beg, beg + deg), with the value sv that relaxes
// its edges.  The wavefront walks the concatenation of the 64 rows 64 edges
// at a time; in each step lane k takes the k-th edge and finds its row by a
// six-step search over the exclusive prefix of the degrees.
template <class F>
__device__ __forceinline__ void wave_rows_balanced(int beg, int deg, int sv, F&& f) {
    const int lane = threadIdx.x & 63;
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63, 64);
    const int excl = incl - deg;
    for (int base = 0; base < total; base += 64) {
        const int k = base + lane;
        int o = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int cand = o + step;
            const int ex = __shfl(excl, cand, 64);
            if (ex <= k) o = cand;
        }
        const int ob = __shfl(beg, o, 64);
        const int oe = __shfl(excl, o, 64);
        const int os = __shfl(sv, o, 64);
        if (k < total) f(ob + (k - oe), os);
    }
}

// ---------------------------------------------------------- algorithms ----

// Relax one edge e (p -> t = col[e]) with the tail's value sv.  Returns true
// when this lane lowered val[t] (the caller pushes t or counts an update).
template <int A>
__device__ __forceinline__ bool relax_edge(const Round& R, const int* col, int e, int sv, int& t) {
    t = col[e];
    int* val = R.val;
    if (A == SSSP) {
        // sv < INF and w >= 0: the sum fits 32 unsigned bits; anything at or
        // above 2^31 cannot beat a stored value and is dropped
        const unsigned cand = (unsigned)sv + (unsigned)R.g.w[e];
        const int cur = val[t];
        if (cand < (unsigned)cur) {
            const int old = atomicMin(&val[t], (int)cand);
            return (int)cand < old;
        }
        return false;
    } else if (A == BFS) {
        const int nl = sv + 1;
        if (val[t] > nl) {
            val[t] = nl;
            return true;
        }
        return false;
    } else {
        const int cur = val[t];
        if (sv < cur) {
            const int old = atomicMin(&val[t], sv);
            return sv < old;
        }
        return false;
    }
}

// Relax U edges per lane with the loads of all of them in flight before the
// first compare: column indices (and weights), then head values, then the
// atomics.  Reading every head value before any atomic of the batch is safe
// because values only decrease.  ok[j] masks the lanes that own an edge.
// ATOM: BFS lowers levels with atomicMin instead of a plain store (needed
// when the tails of one round hold different levels, as under local
// expansion; a plain store could then overwrite a lower level).
template <int A, int U, bool PUSH, bool ATOM = false>
__device__ __forceinline__ void relax_batch(const Round& R, const int* col, const int (&e)[U],
                                            const int (&sv)[U], const bool (&ok)[U], int nxt,
                                            Acc& acc, int bound = kInf) {
    int* val = R.val;
    int t[U], wt[U], cur[U];
#pragma unroll
    for (int j = 0; j < U; ++j) t[j] = ok[j] ? col[e[j]] : 0;
    if (A == SSSP) {
#pragma unroll
        for (int j = 0; j < U; ++j) wt[j] = ok[j] ? R.g.w[e[j]] : 0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) cur[j] = ok[j] ? val[t[j]] : 0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        if (!ok[j]) continue;
        acc.e++;
        // An edge whose loaded head value the candidate beats lowers that
        // head in this round -- by this atomic, or by a concurrent lower one
        // whose lane pushes the head too -- so the push is decided from the
        // load and the atomic returns nothing: the lane does not wait for it
        // (pushes are idempotent flag stores).
        bool hit = false;
        if (A == SSSP) {
            const unsigned cand = (unsigned)sv[j] + (unsigned)wt[j];
            if (cand < (unsigned)cur[j]) {
                atomicMin(&val[t[j]], (int)cand);
                hit = true;
            }
        } else if (A == BFS) {
            const int nl = sv[j] + 1;
            if (cur[j] > nl) {
                if (ATOM)
                    atomicMin(&val[t[j]], nl);
                else
                    val[t[j]] = nl;
                hit = true;
            }
        } else {
            if (sv[j] < cur[j]) {
                atomicMin(&val[t[j]], sv[j]);
                hit = true;
            }
        }
        if (hit) {
            if (PUSH) {
                R.ws.vflag[nxt][t[j]] = 1;
                R.ws.tflag[nxt][t[j] >> 6] = 1;
                acc.p++;
                if (A == CC && R.fedges) acc.add_f(R.g.srow[t[j] + 1] - R.g.srow[t[j]]);
                if (A == SSSP && R.fedges) acc.add_f(R.g.row[t[j] + 1] - R.g.row[t[j]]);
                // near-far: a new distance below the round's bound keeps the
                // bound where it is for the next round
                if (A == SSSP && (unsigned)sv[j] + (unsigned)wt[j] < (unsigned)bound) acc.nr = 1;
            } else {
                acc.u++;
            }
        }
    }
}

// The edges [e0, e1) of one row, all with tail value sv, relaxed by the
// whole wavefront U x 64 edges per step.
template <int A, bool PUSH, int U = kBatch, bool ATOM = false>
__device__ __forceinline__ void wave_relax_range(const Round& R, const int* col, int e0, int e1,
                                                 int sv, int nxt, Acc& acc, int bound = kInf) {
    const int lane = threadIdx.x & 63;
    for (int eb = e0; eb < e1; eb += 64 * U) {
        int e[U], s[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            e[j] = eb + j * 64 + lane;
            ok[j] = e[j] < e1;
            s[j] = sv;
        }
        relax_batch<A, U, PUSH, ATOM>(R, col, e, s, ok, nxt, acc, bound);
    }
}

// Lanes hold one row each, [beg, beg + deg), with tail value sv.  The
// wavefront walks the concatenation of the 64 rows U x 64 edges per
// step; edge k of a step belongs to the row found by a six-step search over
// the exclusive prefix of the degrees.
template <int A, bool PUSH, int U = kBatch>
__device__ __forceinline__ void wave_relax_rows(const Round& R, const int* col, int beg, int deg,
                                                int sv, int nxt, Acc& acc, int bound = kInf) {
    const int lane = threadIdx.x & 63;
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63, 64);
    const int excl = incl - deg;
    for (int base = 0; base < total; base += 64 * U) {
        int e[U], s[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = base + j * 64 + lane;
            int o = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int cand = o + step;
                if (__shfl(excl, cand, 64) <= k) o = cand;
            }
            e[j] = __shfl(beg, o, 64) + (k - __shfl(excl, o, 64));
            s[j] = __shfl(sv, o, 64);
            ok[j] = k < total;
        }
        relax_batch<A, U, PUSH>(R, col, e, s, ok, nxt, acc, bound);
    }
}

// Value and activity of vertex u as the tail of its edges.
//  sync:  SSSP every reached vertex; BFS the vertices of level r; CC all.
//  async: u is on the frontier; SSSP/CC read its current value, BFS uses r.
// For CC the shortcut label[u] = label[label[u]] is applied first (counted as
// an update so that a sweep which only shortcuts is not the last one).
template <int A, bool ASYNC>
__device__ __forceinline__ bool tail_value(const Round& R, int u, int& sv, Acc& acc) {
    int* val = R.val;
    if (A == SSSP) {
        sv = val[u];
        return ASYNC || sv != kInf;
    } else if (A == BFS) {
        sv = R.r;
        return ASYNC || val[u] == R.r;
    } else {
        int x = val[u];
        if (R.jump) {
            const int y = val[x];
            if (y < x) {
                const int old = atomicMin(&val[u], y);
                if (!ASYNC && y < old) acc.u++;
                x = y;
            }
        }
        sv = x;
        return true;
    }
}

__device__ __forceinline__ void push(const Round& R, int nxt, int t) {
    R.ws.vflag[nxt][t] = 1;
    R.ws.tflag[nxt][t >> 6] = 1;
}

// Heavy frontier rows: round r sets row u's bit in hbits[r & 1] (an atomic
// OR that returns nothing) and the chunk kernel of the same round serves the
// chunks of the rows whose bit is set.  The bits fit in the dies' L2 (512 KB
// for 4M vertices), so the chunk kernel's check of every chunk is a cached
// load; the round kernel of round r clears the bits of round r-1 (its chunk
// kernel has completed) so that round r+1 finds them clear.
__device__ __forceinline__ void mark_heavy(const Round& R, int u) {
    atomicOr(&R.ws.hbits[R.r & 1][u >> 5], 1u << (u & 31));
}

__device__ __forceinline__ bool heavy_marked(const Round& R, int u) {
    return (R.ws.hbits[R.r & 1][u >> 5] >> (u & 31)) & 1u;
}

__device__ __forceinline__ void clear_prev_heavy(const Round& R) {
    if (R.g.n_hchunks == 0 && R.g.n_shchunks == 0) return;  // no heavy row to mark
    const long long words = ((long long)R.g.n + 31) / 32;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    unsigned* b = R.ws.hbits[(R.r + 1) & 1];
    for (long long i = tid; i < words; i += tt) b[i] = 0;
}

// ------------------------------------------------------ local expansion ----
// A worklist round with local expansion (Round::hops > 0) lets a wavefront
// serve again, within the same round, the vertices it has just lowered: a
// successful relaxation whose new value is below the round's bound goes,
// with that value, to a list of kLocalCap entries in the wavefront's LDS
// instead of the next frontier, and the wavefront serves the list up to
// `hops` times.  Entries past the capacity, and the list left after the last
// pass, go to the next frontier.  Serving a vertex with the value this lane
// wrote is safe: if another lane lowered it further since, that lane put it
// on a list or the frontier itself.  On a high-diameter graph this advances
// the frontier several steps per launch; the fixpoint is the same.
// The list holds (vertex, value, row begin, row end): the row offsets of a
// head that may be lowered below the bound are loaded together with its
// atomic, so that serving the
// entry in the next pass starts at the column loads -- one dependent load
// fewer per pass.  128 entries per list, served 64 (one per lane) at a time:
// on a grid a served vertex lowers one or two new heads, so a list of 64
// overflowed to the next round at once (grid4096 SSSP: 586 rounds with 64
// entries, 437 with 128 or 256; er23 SSSP 3.47 / 3.40 / 3.29 ms with 64 /
// 128 / 256 two-word entries).
constexpr int kLocalCap = 128;

// Rows of at most kShortRow edges are relaxed one lane per row when a whole
// list of them is served (see wave_relax_rows_local).  grid4096 step: 6.45
// GTEPS with the balanced walk only, 6.68 with 4, 7.03 with 5, 6.42 with 6
// and 6.07 with 8 (lists with a longer row take the balanced walk).
constexpr int kShortRow = 5;

// direct: no head-value load before the atomic (the atomic's returned value
// decides): one round trip fewer per edge, one atomic more per edge that
// would not have lowered its head.  BFS passes over a wavefront's own list
// are always direct (their vertices were just reached and mostly reach new
// heads in turn: grid4096 BFS 13.5 -> 11.6 ms).  SSSP passes are direct
// when Round::direct_lists says so: on a deep graph a round is a chain of
// dependent passes run by few wavefronts, so the round trip saved counts
// and the extra atomics do not (grid4096 step +10%); on shallow graphs the
// rounds are wide and the extra atomics cost more (rmat22 -2%, er23 -4%).
// Choosing per pass from the share of the previous pass's edges that
// lowered their head (direct above one half) gained nothing on grid4096.
// The atomics of a lane's U edges are all issued before the first returned
// value is looked at (then the ballots and list writes), so their round
// trips overlap instead of following one another.
template <int A, int U>
__device__ __forceinline__ void relax_batch_local(const Round& R, const int* row, const int* col,
                                                  const int (&e)[U], const int (&sv)[U],
                                                  const bool (&ok)[U], int nxt, Acc& acc,
                                                  int bound, int4* lst, int& ln, bool direct) {
    int* val = R.val;
    const int lane = threadIdx.x & 63;
    int t[U], wt[U], cur[U], nv[U], old[U], rb[U], re[U];
#pragma unroll
    for (int j = 0; j < U; ++j) t[j] = ok[j] ? col[e[j]] : 0;
    if (A == SSSP) {
#pragma unroll
        for (int j = 0; j < U; ++j) wt[j] = ok[j] ? R.g.w[e[j]] : 0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) cur[j] = ok[j] && !direct ? val[t[j]] : kInf;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        nv[j] = 0;
        old[j] = 0;  // no atomic: counts as no decrease
        rb[j] = re[j] = 0;
        if (ok[j]) {
            acc.e++;
            bool go;
            if (A == SSSP) {
                const unsigned cand = (unsigned)sv[j] + (unsigned)wt[j];
                go = cand < (unsigned)cur[j];
                nv[j] = (int)cand;
            } else {
                nv[j] = A == BFS ? sv[j] + 1 : sv[j];
                go = nv[j] < cur[j];
            }
            if (go) {
                // only a head below the bound can go to the list
                if (nv[j] < bound) {
                    rb[j] = row[t[j]];
                    re[j] = row[t[j] + 1];
                }
                old[j] = atomicMin(&val[t[j]], nv[j]);
            } else {
                old[j] = nv[j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const bool hit = ok[j] && nv[j] < old[j];
        const bool keep = hit && nv[j] < bound;
        const unsigned long long km = __ballot(keep);
        const int pos = ln + __popcll(km & ((1ull << lane) - 1));
        if (keep && pos < kLocalCap) {
            lst[pos] = make_int4(t[j], nv[j], rb[j], re[j]);
        } else if (hit) {
            push(R, nxt, t[j]);
            acc.p++;
            if (nv[j] < bound) acc.nr = 1;
        }
        ln = min(ln + __popcll(km), kLocalCap);
    }
}

// wave_relax_rows with relax_batch_local, or one lane per row when every
// row of the list is short.
template <int A, int U>
__device__ __forceinline__ void wave_relax_rows_local(const Round& R, const int* row,
                                                      const int* col, int beg, int deg, int sv,
                                                      int nxt, Acc& acc, int bound, int4* lst,
                                                      int& ln, bool direct) {
    const int lane = threadIdx.x & 63;
    if (__ballot(deg > kShortRow) == 0) {
        // every row has at most kShortRow edges: each lane relaxes its own
        // row, all its edges in flight at once, with no scan and no search.
        // A pass over a list is one step of the chain of dependent passes a
        // round of a deep graph waits for, and the shuffles of the scan and
        // the search are a good part of a pass over short rows.
        int e[kShortRow], s[kShortRow];
        bool ok[kShortRow];
#pragma unroll
        for (int j = 0; j < kShortRow; ++j) {
            e[j] = beg + j;
            s[j] = sv;
            ok[j] = j < deg;
        }
        relax_batch_local<A, kShortRow>(R, row, col, e, s, ok, nxt, acc, bound, lst, ln, direct);
        return;
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63, 64);
    const int excl = incl - deg;
    for (int base = 0; base < total; base += 64 * U) {
        int e[U], s[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = base + j * 64 + lane;
            int o = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int cand = o + step;
                if (__shfl(excl, cand, 64) <= k) o = cand;
            }
            e[j] = __shfl(beg, o, 64) + (k - __shfl(excl, o, 64));
            s[j] = __shfl(sv, o, 64);
            ok[j] = k < total;
        }
        relax_batch_local<A, U>(R, row, col, e, s, ok, nxt, acc, bound, lst, ln, direct);
    }
}

// ------------------------------------------------------------ kernels ----

// Init: values INF (labels = ids for CC), the source at 0 and on the first
// frontier.  A multi-source traversal (R.nsrc > 0) marks no source here;
// k_seed does it after this kernel.
__global__ __launch_bounds__(256) void k_init(Round R, int algo, int async) {
    const int n = R.g.n;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    const long long src = R.nsrc > 0 ? -1 : R.source;
    for (long long v = tid; v < n; v += tt) {
        R.val[v] = algo == CC ? (int)v : (v == src ? 0 : kInf);
        if (R.rmin) R.rmin[v] = kInf;
        if (async) {
            const bool on = algo == CC || v == src;
            R.ws.vflag[0][v] = on;
            R.ws.vflag[1][v] = 0;
            if ((v & 63) == 0) {
                const long long t = v >> 6;
                R.ws.tflag[0][t] = algo == CC || t == (src >> 6);
                R.ws.tflag[1][t] = 0;
            }
        }
    }
    if (async) {
        const long long words = ((long long)n + 31) / 32;
        for (long long i = tid; i < words; i += tt) R.ws.hbits[0][i] = R.ws.hbits[1][i] = 0;
    }
    for (long long i = tid; i < kKinds * kMaxStatBlocks; i += tt) R.ws.stat[i] = Stat{0, 0, 0, 0, 0};
    if (tid == 0) *R.ws.ctl = Ctl{};
}

// Sources of a multi-source traversal (disjoint instances packed into one
// graph): value 0 and a place on the first frontier.
__global__ __launch_bounds__(256) void k_seed(Round R, int async) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long i = tid; i < R.nsrc; i += tt) {
        const int s = R.sources[i];
        R.val[s] = 0;
        if (async) {
            R.ws.vflag[0][s] = 1;
            R.ws.tflag[0][s >> 6] = 1;
        }
    }
}

// Synchronous vertex sweep (Algorithm 1; Algorithm 3 for BFS).
template <int A, int MAP>
__global__ __launch_bounds__(256) void k_vsync(Round R) {
    if (!round_begin(R)) return;
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int n = g.n;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    Acc acc;

    if (MAP == MAP_BALANCED) {
        const int2* hch = A == CC ? g.shchunks : g.hchunks;
        const long long nh = A == CC ? g.n_shchunks : g.n_hchunks;
        for (long long it = gw; it < nh + ntiles; it += tw) {
            if (it < nh) {
                const int2 hc = hch[it];
                const int u = hc.x;
                const int e1 = min(hc.y + g.chunk, row[u + 1]);
                int sv;
                if (tail_value<A, false>(R, u, sv, acc)) {
                    if (lane == 0) acc.v++;
                    wave_relax_range<A, false>(R, col, hc.y, e1, sv, 0, acc);
                }
            } else {
                const int u = (int)((it - nh) * 64 + lane);
                int beg = 0, deg = 0, sv = 0;
                if (u < n) {
                    const int rb = row[u], re = row[u + 1];
                    if (re - rb <= g.heavy && tail_value<A, false>(R, u, sv, acc)) {
                        beg = rb;
                        deg = re - rb;
                        acc.v++;
                    }
                }
                wave_relax_rows<A, false>(R, col, beg, deg, sv, 0, acc);
            }
        }
    } else if (MAP == MAP_THREAD) {
        const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        const long long tt = (long long)gridDim.x * blockDim.x;
        for (long long uu = tid; uu < n; uu += tt) {
            const int u = (int)uu;
            int sv;
            if (!tail_value<A, false>(R, u, sv, acc)) continue;
            acc.v++;
            const int re = row[u + 1];
            for (int e = row[u]; e < re; ++e) {
                int t;
                acc.e++;
                if (relax_edge<A>(R, col, e, sv, t)) acc.u++;
            }
        }
    } else {  // MAP_WAVE
        for (long long uu = gw; uu < n; uu += tw) {
            const int u = (int)uu;
            int sv;
            if (!tail_value<A, false>(R, u, sv, acc)) continue;
            if (lane == 0) acc.v++;
            const int re = row[u + 1];
            for (int e = row[u] + lane; e < re; e += 64) {
                int t;
                acc.e++;
                if (relax_edge<A>(R, col, e, sv, t)) acc.u++;
            }
        }
    }
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// One edge of the synchronous edge sweep (Algorithm 2; the edge form of
// Algorithm 3 for BFS; CC relaxes both directions of a stored edge unless
// the input is symmetric, where the reverse edge is stored too).
// A CC sweep of the per-round schedule also puts every vertex it lowers on
// the next round's frontier, with the vertex's row length counted.
__device__ __forceinline__ void sweep_push(const Round& R, int x, Acc& acc) {
    const int nxt = (R.r & 1) ^ 1;
    R.ws.vflag[nxt][x] = 1;
    R.ws.tflag[nxt][x >> 6] = 1;
    acc.p++;
    acc.add_f(R.g.srow[x + 1] - R.g.srow[x]);
}

typedef int v4i __attribute__((ext_vector_type(4)));

// Lower a CC label in an edge sweep.  Sweeps of the per-round schedule
// (PUSH), whose later worklist rounds revisit only the pushed vertices, use
// an atomic minimum so that no decrease is lost.  Plain sweeps store: two
// lanes storing into one label at once can lose the lower value, but the
// label keeps a value that some edge carried (never above the vertex's own
// id), that edge stays inconsistent and a later sweep lowers it again.
// Plain sweeps end after a sweep in which no lane stored anything, which saw
// every edge consistent: each component then holds one label, the id of one
// of its vertices and no larger than any of them -- the smallest.  Every
// device-scope atomic sends its write on to memory (32 bytes of write
// traffic each by the counters), where stores stay in the die's cache until
// the sweep ends, and a first sweep lowers labels across half of the edges
// (er23 CC: 3.10 ms with atomics, 2.59 ms with stores).
template <bool PUSH>
__device__ __forceinline__ void cc_lower(int* p, int x) {
    if (PUSH) atomicMin(p, x);
    else *p = x;
}

template <int A, bool PUSH = false>
__device__ __forceinline__ void edge_sync_one(const Round& R, int u, int t, int e, Acc& acc) {
    int* val = R.val;
    acc.e++;
    if (A == SSSP) {
        const int du = val[u];
        if (du == kInf) return;
        const unsigned cand = (unsigned)du + (unsigned)R.g.w[e];
        if (cand < (unsigned)val[t]) {
            const int old = atomicMin(&val[t], (int)cand);
            if ((int)cand < old) acc.u++;
        }
    } else if (A == BFS) {
        const int lev = R.r;
        if (val[u] == lev && val[t] > lev + 1) {
            val[t] = lev + 1;
            acc.u++;
        }
    } else {
        // CC: lowered without a returned value (see edge_sync_four)
        const int lu = val[u], lt = val[t];
        if (lu < lt) {
            cc_lower<PUSH>(&val[t], lu);
            acc.u++;
            if (PUSH) sweep_push(R, t, acc);
        } else if (lt < lu && !R.g.symmetric) {
            cc_lower<PUSH>(&val[u], lt);
            acc.u++;
            if (PUSH) sweep_push(R, u, acc);
        }
    }
}

// Four consecutive edges [e, e+4) of an edge list (16-byte aligned), with
// every value loaded before the first atomic.
template <int A, bool PUSH = false>
__device__ __forceinline__ void edge_sync_four(const Round& R, const int* src, const int* col,
                                               const int* w, long long e, Acc& acc) {
    const DevGraph& g = R.g;
    int* val = R.val;
    {
        // the edge arrays stream through once per sweep: non-temporal
        // loads leave the L2 to the values they index (er23 step +1.4%,
        // grid4096 CC sweeps 2.59 -> 2.42 ms)
        const v4i s4 = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(src + e));
        const v4i c4 = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(col + e));
        const int u[4] = {s4.x, s4.y, s4.z, s4.w};
        const int t[4] = {c4.x, c4.y, c4.z, c4.w};
        int wt[4] = {0, 0, 0, 0};
        if (A == SSSP) {
            const v4i w4 = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(w + e));
            wt[0] = w4.x;
            wt[1] = w4.y;
            wt[2] = w4.z;
            wt[3] = w4.w;
        }
        // every value of the four edges is loaded before the first atomic;
        // a head value is loaded only when the tail can relax the edge
        int vu[4], vt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) vu[j] = val[u[j]];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool need = A == SSSP ? vu[j] != kInf : A == BFS ? vu[j] == R.r : true;
            vt[j] = need ? val[t[j]] : 0;
        }
        acc.e += 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (A == SSSP) {
                if (vu[j] == kInf) continue;
                const unsigned cand = (unsigned)vu[j] + (unsigned)wt[j];
                if (cand < (unsigned)vt[j] && (int)cand < atomicMin(&val[t[j]], (int)cand)) acc.u++;
            } else if (A == BFS) {
                if (vu[j] == R.r && vt[j] > R.r + 1) {
                    val[t[j]] = R.r + 1;
                    acc.u++;
                }
            } else {
                // CC sweeps lower labels without waiting for a returned
                // value: a lane whose loads show a lower label on one end
                // counts the change (and pushes the other end) itself, and a
                // sweep that reports no change saw every edge consistent.
                // (Most edges of a first sweep lower a label: er23's first
                // sweep took 2.25 ms with returning atomics, 2.0 ms with
                // atomics that return nothing.)
                if (vu[j] < vt[j]) {
                    cc_lower<PUSH>(&val[t[j]], vu[j]);
                    acc.u++;
                    if (PUSH) sweep_push(R, t[j], acc);
                } else if (vt[j] < vu[j] && !g.symmetric) {
                    cc_lower<PUSH>(&val[u[j]], vt[j]);
                    acc.u++;
                    if (PUSH) sweep_push(R, u[j], acc);
                }
            }
        }
    }
}

// Synchronous edge sweep.  With the head-partitioned edge list, block b
// sweeps part b % kXcd: workgroups are dispatched to the accelerator dies
// round-robin, so each die gathers and updates the values of one slice of
// the vertices only, and that slice stays in the die's own L2.  (Any grid
// size is correct; a grid that is not a multiple of kXcd walks all parts.)
template <int A, bool PUSH>
__device__ __forceinline__ void esync_body(const Round& R, Acc& acc) {
    const DevGraph& g = R.g;
    if (g.psrc) {
        const bool split = gridDim.x >= kXcd && gridDim.x % kXcd == 0;
        const int p0 = split ? (int)(blockIdx.x % kXcd) : 0;
        const int p1 = split ? p0 + 1 : kXcd;
        const long long bpp = split ? gridDim.x / kXcd : gridDim.x;
        const long long bi = split ? blockIdx.x / kXcd : blockIdx.x;
        for (int p = p0; p < p1; ++p) {
            const long long e1 = g.poff[p + 1];
            for (long long e = g.poff[p] + (bi * blockDim.x + threadIdx.x) * 4; e < e1;
                 e += bpp * blockDim.x * 4)
                edge_sync_four<A, PUSH>(R, g.psrc, g.pcol, g.pw, e, acc);
        }
    } else {
        const int m = g.m;
        const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        const long long tt = (long long)gridDim.x * blockDim.x;
        const int m4 = m & ~3;
        for (long long e = tid * 4; e < m4; e += tt * 4)
            edge_sync_four<A, PUSH>(R, g.src, g.col, g.w, e, acc);
        for (long long e = m4 + tid; e < m; e += tt)
            edge_sync_one<A, PUSH>(R, g.src[e], g.col[e], (int)e, acc);
    }
}

// Round 0 of the per-round CC schedule.  Labels start as the vertex ids, so
// one synchronous step is label[v] = min(v, smallest neighbour id): a
// segmented minimum over the both-directions rows that reads the column
// indices only -- no label gathers, and no atomics except one per heavy-row
// chunk.  Light rows: a wavefront takes a tile of 64 rows, walks their edges
// with the balanced mapping and reduces per row in LDS.  Heavy rows: one
// wavefront per heavy-row chunk, one atomic minimum per chunk.  Every vertex
// whose label drops is pushed (with its row length counted), as a sweep
// does.  (An in-place edge sweep carries labels further than this one
// synchronous step, so the plain sweep schedule keeps its first sweep: on a
// uniform graph the step costs it one extra sweep.)
__device__ void cc_first_pass(const Round& R, Acc& acc) {
    const DevGraph& g = R.g;
    const int n = g.n;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    __shared__ int s_min[4][64];  // blocks of 256 threads: four wavefronts
    int* smin = s_min[threadIdx.x >> 6];
    for (long long t = gw; t < ntiles; t += tw) {
        const int v = (int)(t * 64 + lane);
        int rb = 0, deg = 0;
        if (v < n) {
            rb = g.srow[v];
            deg = g.srow[v + 1] - rb;
        }
        const bool light = deg <= g.heavy;
        smin[lane] = v;
        __builtin_amdgcn_wave_barrier();
        wave_rows_balanced(rb, light ? deg : 0, lane,
                           [&](int e, int slot) { atomicMin(&smin[slot], g.scol[e]); });
        __builtin_amdgcn_wave_barrier();
        if (v < n && light) {
            const int x = smin[lane];
            acc.e += deg;
            if (x < v) {
                R.val[v] = x;
                acc.u++;
                sweep_push(R, v, acc);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // Heavy rows, chunk by chunk (kChunk edges, the chunk size of every
    // graph).  The loop is pipelined across a wavefront's chunks: the next
    // chunk's descriptor and row end are fetched while this chunk's columns
    // load; the column loads of a chunk are issued together and need only
    // the chunk's first edge (indices clamped to the column array, lanes
    // past the row end masked after the load); and the result of a chunk's
    // atomicMin (did it lower the label: push the row) is read one chunk
    // later, so that the atomic's round trip overlaps the next chunk's loads.
    constexpr int C = kChunk / 64;
    const long long nch = g.n_shchunks;
    const int last = g.ms - 1;
    long long k = gw;
    int2 c = k < nch ? g.shchunks[k] : make_int2(0, 0);
    int rend = k < nch ? g.srow[c.x + 1] : 0;
    int prow = -1, pold = 0, px = 0;  // lane 0: the previous chunk's atomic
    for (; k < nch; k += tw) {
        const long long kn = k + tw;
        const int2 cn = kn < nch ? g.shchunks[kn] : c;
        int v[C];
#pragma unroll
        for (int j = 0; j < C; ++j) v[j] = g.scol[min(c.y + j * 64 + lane, last)];
        const int e1 = min(c.y + kChunk, rend);
        int x = kInf;
#pragma unroll
        for (int j = 0; j < C; ++j)
            if (c.y + j * 64 + lane < e1) x = min(x, v[j]);
        const int rendn = kn < nch ? g.srow[cn.x + 1] : 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) x = min(x, __shfl_xor(x, d, 64));
        if (lane == 0) {
            if (prow >= 0 && px < pold) {
                acc.u++;
                sweep_push(R, prow, acc);
            }
            acc.e += e1 - c.y;
            pold = atomicMin(&R.val[c.x], x);
            px = x;
            prow = c.x;
        }
        c = cn;
        rend = rendn;
    }
    if (lane == 0 && prow >= 0 && px < pold) {
        acc.u++;
        sweep_push(R, prow, acc);
    }
}

template <int A>
__global__ __launch_bounds__(256) void k_esync(Round R) {
    if (!round_begin(R)) return;
    Acc acc;
    esync_body<A, false>(R, acc);
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Asynchronous vertex round: the frontier of round r is the set of flagged
// vertices; each wavefront scans 64 tile flags at a time and serves the
// flagged tiles it finds.
// Serve the np vertices listed in pend[0, np) of this wavefront (lane k takes
// entry k): the tail value, far vertices of the near-far schedule back onto
// the frontier, heavy rows marked for the chunk kernel, light rows walked by
// the balanced mapping.
template <int A, int U>
__device__ __forceinline__ void serve_list(const Round& R, const int* row, const int* col,
                                           const int* pend, int np, int nxt, bool nf, int bound,
                                           Acc& acc) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    const int u = lane < np ? pend[lane] : -1;
    __builtin_amdgcn_wave_barrier();
    bool on = u >= 0;
    int rb = 0, re = 0, sv = 0;
    if (on) {
        tail_value<A, true>(R, u, sv, acc);
        rb = row[u];
        re = row[u + 1];
        // a far vertex waits on the frontier for a later bound (with
        // far_degree > 0 only its long rows wait; short ones go now)
        const bool defer = nf && sv >= bound && (R.far_degree == 0 || re - rb > R.far_degree);
        if (defer) {
            push(R, nxt, u);
            on = false;
        }
        // counted without a branch: incrementing one of two counters
        // under a condition made the compiler keep them in scratch memory
        acc.u += defer;
        acc.v += !defer;
    }
    const bool hv = on && re - rb > R.g.heavy;
    if (hv) mark_heavy(R, u);
    wave_relax_rows<A, true, U>(R, col, on && !hv ? rb : 0, on && !hv ? re - rb : 0, sv, nxt, acc,
                                bound);
}

// Balanced worklist round with the frontier packed per wavefront: the
// wavefront collects the flagged vertices of the tiles it scans into a
// 64-entry list in LDS and serves a full list at a time.  (A tile of a
// sparse frontier holds a few flagged vertices; serving the tiles one by one
// leaves most lanes idle in every step of the edge walk.)
template <int A, int U>
__device__ __forceinline__ void vasync_packed(const Round& R, Acc& acc, bool nf, int bound) {
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int n = g.n;
    const int cur = R.r & 1, nxt = cur ^ 1;
    unsigned char* vf = R.ws.vflag[cur];
    unsigned char* tf = R.ws.tflag[cur];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    const long long nitems = (ntiles + 63) / 64 * kParts;
    __shared__ int s_pend[4][64];  // blocks of 256 threads: four wavefronts
    int* pend = s_pend[threadIdx.x >> 6];
    int np = 0;  // vertices in the list (the same in every lane)
    for (long long it = gw; it < nitems; it += tw) {
        const long long st = it / kParts;
        const int part = (int)(it % kParts);
        const long long t = st * 64 + lane;
        const bool mine = lane / (64 / kParts) == part;
        const bool tfl = mine && t < ntiles && tf[t] != 0;
        unsigned long long tm = __ballot(tfl);
        if (tfl) tf[t] = 0;
        while (tm) {
            const int b = __ffsll(tm) - 1;
            tm &= tm - 1;
            const int u = (int)((st * 64 + b) * 64 + lane);
            const bool on = u < n && vf[u] != 0;
            if (on) vf[u] = 0;
            const unsigned long long om = __ballot(on);
            const int c = __popcll(om);
            if (np + c > 64) {
                serve_list<A, U>(R, row, col, pend, np, nxt, nf, bound, acc);
                np = 0;
            }
            if (on) pend[np + __popcll(om & ((1ull << lane) - 1))] = u;
            np += c;
        }
    }
    if (np > 0) serve_list<A, U>(R, row, col, pend, np, nxt, nf, bound, acc);
}

template <int A, int MAP, int U = batch_for(A, false)>
__device__ __forceinline__ void vasync_body(const Round& R, Acc& acc, bool nf, int bound) {
    if (MAP == MAP_BALANCED) {
        vasync_packed<A, U>(R, acc, nf, bound);
        return;
    }
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int n = g.n;
    const int cur = R.r & 1, nxt = cur ^ 1;
    unsigned char* vf = R.ws.vflag[cur];
    unsigned char* tf = R.ws.tflag[cur];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    const long long nitems = (ntiles + 63) / 64 * kParts;
    for (long long it = gw; it < nitems; it += tw) {
        const long long st = it / kParts;
        const int part = (int)(it % kParts);
        const long long t = st * 64 + lane;
        const bool mine = lane / (64 / kParts) == part;
        const bool tfl = mine && t < ntiles && tf[t] != 0;
        unsigned long long tm = __ballot(tfl);
        if (tfl) tf[t] = 0;
        while (tm) {
            const int b = __ffsll(tm) - 1;
            tm &= tm - 1;
            const int u = (int)((st * 64 + b) * 64 + lane);
            bool on = u < n && vf[u] != 0;
            if (on) vf[u] = 0;
            int rb = 0, re = 0, sv = 0;
            if (on) {
                tail_value<A, true>(R, u, sv, acc);
                // a far vertex waits on the frontier for a later bound
                const bool defer = nf && sv >= bound;
                if (defer) {
                    push(R, nxt, u);
                    on = false;
                } else {
                    rb = row[u];
                    re = row[u + 1];
                }
                acc.u += defer;
                acc.v += !defer;
            }
            if (MAP == MAP_THREAD) {
                if (on)
                    for (int e = rb; e < re; ++e) {
                        int t2;
                        acc.e++;
                        if (relax_edge<A>(R, col, e, sv, t2)) {
                            push(R, nxt, t2);
                            acc.p++;
                        }
                    }
            } else {  // MAP_WAVE: the wavefront serves its flagged rows in turn
                unsigned long long am = __ballot(on);
                while (am) {
                    const int o = __ffsll(am) - 1;
                    am &= am - 1;
                    const int ob = __shfl(rb, o, 64), oe = __shfl(re, o, 64);
                    const int os = __shfl(sv, o, 64);
                    for (int e = ob + lane; e < oe; e += 64) {
                        int t2;
                        acc.e++;
                        if (relax_edge<A>(R, col, e, os, t2)) {
                            push(R, nxt, t2);
                            acc.p++;
                        }
                    }
                }
            }
        }
    }
}

// NF: the near-far schedule (SSSP, balanced mapping, R.delta > 0); a
// separate instantiation keeps its bookkeeping out of the plain rounds.
template <int A, int MAP, bool NF = false>
__global__ __launch_bounds__(256) void k_vasync(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    const bool nf = NF;
    const int bound = nf ? nearfar_bound(R) : kInf;
    Acc acc;
    vasync_body<A, MAP, batch_for(A, NF)>(R, acc, nf, bound);
    if (nf) nearfar_finish(R, acc);
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// serve_list under local expansion: the frontier vertices in pend (their
// current values read here; BFS too, since levels differ within a round),
// then up to R.hops passes over the wavefront's own list.  lb holds two
// lists of kLocalCap (vertex, value, row begin, row end) entries that the
// passes alternate.
template <int A, int U>
__device__ __forceinline__ void serve_local(const Round& R, const int* row, const int* col,
                                            const int* pend, int np, int nxt, bool nf, int bound,
                                            Acc& acc, int4* lb) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    int u = lane < np ? pend[lane] : -1;
    __builtin_amdgcn_wave_barrier();
    bool on = u >= 0;
    int rb = 0, re = 0, sv = 0;
    if (on) {
        if (A == BFS) sv = R.val[u];
        else tail_value<A, true>(R, u, sv, acc);
        rb = row[u];
        re = row[u + 1];
        const bool defer = nf && sv >= bound && (R.far_degree == 0 || re - rb > R.far_degree);
        if (defer) {
            push(R, nxt, u);
            on = false;
        }
        acc.u += defer;  // without a branch, as in serve_list
        acc.v += !defer;
    }
    bool hv = on && re - rb > R.g.heavy;
    if (hv) mark_heavy(R, u);
    int ln = 0;
    wave_relax_rows_local<A, U>(R, row, col, on && !hv ? rb : 0, on && !hv ? re - rb : 0, sv,
                                nxt, acc, bound, lb, ln, false);
    const bool direct = A == BFS || (A == SSSP && R.direct_lists);
    for (int pass = 1; ln > 0; ++pass) {
        const int4* cur = lb + ((pass - 1) & 1) * kLocalCap;
        int4* nx = lb + (pass & 1) * kLocalCap;
        const int cn = ln;
        ln = 0;
        // the list is served 64 entries (one per lane) at a time
        for (int base = 0; base < cn; base += 64) {
            __builtin_amdgcn_wave_barrier();
            const int4 x = base + lane < cn ? cur[base + lane] : make_int4(-1, 0, 0, 0);
            __builtin_amdgcn_wave_barrier();
            if (pass > R.hops) {
                // out of passes: the list goes to the next frontier
                if (x.x >= 0) {
                    push(R, nxt, x.x);
                    acc.p++;
                    acc.nr = 1;
                }
                continue;
            }
            u = x.x;
            sv = x.y;
            on = u >= 0;
            rb = x.z;  // loaded with the atomic that put u on the list
            re = x.w;
            if (on) acc.v++;
            hv = on && re - rb > R.g.heavy;
            if (hv) mark_heavy(R, u);
            wave_relax_rows_local<A, U>(R, row, col, on && !hv ? rb : 0,
                                        on && !hv ? re - rb : 0, sv, nxt, acc, bound, nx, ln,
                                        direct);
        }
        if (pass > R.hops) break;
    }
}

// vasync_packed with serve_local.
template <int A, int U>
__device__ __forceinline__ void vasync_local(const Round& R, Acc& acc, bool nf, int bound) {
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int n = g.n;
    const int cur = R.r & 1, nxt = cur ^ 1;
    unsigned char* vf = R.ws.vflag[cur];
    unsigned char* tf = R.ws.tflag[cur];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    const long long nitems = (ntiles + 63) / 64 * kParts;
    __shared__ int s_pend[4][64];  // blocks of 256 threads: four wavefronts
    __shared__ int4 s_loc[4][2 * kLocalCap];
    int* pend = s_pend[threadIdx.x >> 6];
    int4* lb = s_loc[threadIdx.x >> 6];
    int np = 0;
    for (long long it = gw; it < nitems; it += tw) {
        const long long st = it / kParts;
        const int part = (int)(it % kParts);
        const long long t = st * 64 + lane;
        const bool mine = lane / (64 / kParts) == part;
        const bool tfl = mine && t < ntiles && tf[t] != 0;
        unsigned long long tm = __ballot(tfl);
        if (tfl) tf[t] = 0;
        while (tm) {
            const int b = __ffsll(tm) - 1;
            tm &= tm - 1;
            const int u = (int)((st * 64 + b) * 64 + lane);
            const bool on = u < n && vf[u] != 0;
            if (on) vf[u] = 0;
            const unsigned long long om = __ballot(on);
            const int c = __popcll(om);
            if (np + c > 64) {
                serve_local<A, U>(R, row, col, pend, np, nxt, nf, bound, acc, lb);
                np = 0;
            }
            if (on) pend[np + __popcll(om & ((1ull << lane) - 1))] = u;
            np += c;
        }
    }
    if (np > 0) serve_local<A, U>(R, row, col, pend, np, nxt, nf, bound, acc, lb);
}

// Worklist round with local expansion (balanced mapping; NF: near-far).
// At most 80 VGPRs (six wavefronts per SIMD): the near-far form otherwise
// takes 81 and launches 1,280 resident blocks instead of 1,536.
template <int A, bool NF>
__global__ __launch_bounds__(256, 6) void k_vlocal(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    const int bound = NF ? nearfar_bound(R) : kInf;
    Acc acc;
    // the plain rounds' edges in flight: eight (near-far) spill here
    vasync_local<A, batch_for(A, false)>(R, acc, NF, bound);
    if (NF) nearfar_finish(R, acc);
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Asynchronous edge round: for every flagged tile the wavefront walks the
// tile's edge-list range lane by lane (one lane per edge, source from the
// edge list) and relaxes the edges whose source is on the frontier.  Runs of
// light rows are walked; heavy flagged rows go to the chunk queue.
template <int A>
__global__ __launch_bounds__(256) void k_easync(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int* src = A == CC ? g.ssrc : g.src;
    const int n = g.n;
    const int cur = R.r & 1, nxt = cur ^ 1;
    unsigned char* vf = R.ws.vflag[cur];
    unsigned char* tf = R.ws.tflag[cur];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    const long long nitems = (ntiles + 63) / 64 * kParts;
    Acc acc;
    for (long long it = gw; it < nitems; it += tw) {
        const long long st = it / kParts;
        const int part = (int)(it % kParts);
        const long long t = st * 64 + lane;
        const bool mine = lane / (64 / kParts) == part;
        const bool tfl = mine && t < ntiles && tf[t] != 0;
        unsigned long long tm = __ballot(tfl);
        if (tfl) tf[t] = 0;
        while (tm) {
            const int b = __ffsll(tm) - 1;
            tm &= tm - 1;
            const int base_v = (int)((st * 64 + b) * 64);
            const int u = base_v + lane;
            const bool in = u < n;
            const bool on = in && vf[u] != 0;
            if (on) vf[u] = 0;
            int rb = 0, re = 0, sv = 0;
            if (in) {
                rb = row[u];
                re = row[u + 1];
            }
            if (on) {
                tail_value<A, true>(R, u, sv, acc);
                acc.v++;
            }
            const bool light = in && re - rb <= g.heavy;
            // heavy rows are served by the chunk kernel of this round
            if (on && !light) mark_heavy(R, u);
            const unsigned long long am = __ballot(on && light);
            if (am == 0) continue;
            // walk maximal runs of light rows that contain a flagged row
            unsigned long long lm = __ballot(light);
            while (lm) {
                const int a = __ffsll(lm) - 1;
                const unsigned long long rest = ~(lm >> a);
                const int len = rest == 0 ? 64 - a : __ffsll(rest) - 1;
                const unsigned long long run = (len == 64 ? ~0ull : ((1ull << len) - 1)) << a;
                lm &= ~run;
                if ((am & run) == 0) continue;
                const int e0 = __shfl(rb, a, 64);
                const int e1 = __shfl(re, a + len - 1, 64);
                for (int eb = e0; eb < e1; eb += 64 * kBatch) {
                    int e[kBatch], bit[kBatch], os[kBatch];
                    bool act[kBatch];
#pragma unroll
                    for (int j = 0; j < kBatch; ++j) {
                        e[j] = eb + j * 64 + lane;
                        bit[j] = e[j] < e1 ? src[e[j]] - base_v : 0;
                    }
#pragma unroll
                    for (int j = 0; j < kBatch; ++j) {
                        act[j] = e[j] < e1 && ((am >> bit[j]) & 1);
                        // the tail's value is held by the lane of that vertex
                        os[j] = __shfl(sv, bit[j], 64);
                    }
                    relax_batch<A, kBatch, true>(R, col, e, os, act, nxt, acc);
                }
            }
        }
    }
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Direction-optimizing BFS round.  Level r is pushed from the frontier (as in
// k_vasync: out-edges of the flagged vertices, heavy rows to the chunk kernel)
// while the frontier is small, and pulled while it is large: every unvisited
// vertex scans its in-neighbours (the innbrs iterator of the DSL) and takes
// level r+1 at the first one on level r, so no atomics and few edges.  The
// frontier size is the sum of the previous round's per-block push counts;
// every block computes the same sum, so the direction is grid-uniform.
__global__ __launch_bounds__(256) void k_bfs_diropt(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    const DevGraph& g = R.g;
    Ctl* ctl = R.ws.ctl;
    const int n = g.n;
    const int lev = R.r;
    const long long front = R.r > 0 ? prev_front(R) : 1;  // round 0: the source
    const bool pull = front * kPullRatio > n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->pull[R.r % 3] = pull;
        ctl->hgrid[R.r % 3] = 0;  // a push round's heavy kernel rewrites it
    }
    const int cur = R.r & 1, nxt = cur ^ 1;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    Acc acc;
    if (!pull) {
        // push: the balanced frontier round of k_vasync
        vasync_packed<BFS, batch_for(BFS, false)>(R, acc, false, kInf);
    } else {
        // pull: one tile of 64 vertices per wavefront step; the frontier flags
        // of this round are cleared on the way (they are not read)
        unsigned char* vf = R.ws.vflag[cur];
        unsigned char* tf = R.ws.tflag[cur];
        int* val = R.val;
        for (long long t = gw; t < ntiles; t += tw) {
            const int v = (int)(t * 64 + lane);
            const bool in = v < n;
            if (in) vf[v] = 0;
            if (lane == 0) tf[t] = 0;
            const bool todo = in && val[v] == kInf;
            int ib = 0, ie = 0;
            if (todo) {
                // in-neighbours: the whole row of a symmetric graph, else the
                // part of the both-directions row after v's out-edges
                if (g.symmetric) {
                    ib = g.row[v];
                    ie = g.row[v + 1];
                } else {
                    ib = g.srow[v] + (g.row[v + 1] - g.row[v]);
                    ie = g.srow[v + 1];
                }
                acc.v++;
            }
            const int* icol = g.symmetric ? g.col : g.scol;
            bool found = false;
            // short lists: each lane walks its own, kBatch entries at a time
            const bool shortl = todo && ie - ib <= 64;
            for (int e = ib; shortl && !found && e < ie; e += kBatch) {
                int x[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch; ++j) x[j] = e + j < ie ? val[icol[e + j]] : kInf;
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    if (e + j < ie) acc.e++;
                    found |= x[j] == lev;
                }
            }
            // long lists: the wavefront walks them one vertex at a time
            unsigned long long lm = __ballot(todo && !shortl);
            while (lm) {
                const int o = __ffsll(lm) - 1;
                lm &= lm - 1;
                const int ob = __shfl(ib, o, 64), oe = __shfl(ie, o, 64);
                bool hit = false;
                for (int e = ob; e < oe && !hit; e += 64) {
                    const bool h = e + lane < oe && val[icol[e + lane]] == lev;
                    if (e + lane < oe) acc.e++;
                    hit = __ballot(h) != 0;
                }
                if (lane == o) found = hit;
            }
            if (found) {
                val[v] = lev + 1;
                R.ws.vflag[nxt][v] = 1;
                R.ws.tflag[nxt][v >> 6] = 1;
                acc.p++;
            }
        }
    }
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Clear frontier generation `gen` (vertex and tile flags; the arrays are
// padded to whole groups of 64 tiles, 16-byte aligned).
__device__ __forceinline__ void clear_generation(const Round& R, int gen) {
    const long long groups = ((long long)R.g.n + 4095) / 4096;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    uint4* vf = reinterpret_cast<uint4*>(R.ws.vflag[gen]);
    uint4* tf = reinterpret_cast<uint4*>(R.ws.tflag[gen]);
    for (long long i = tid; i < groups * 256; i += tt) vf[i] = make_uint4(0, 0, 0, 0);
    for (long long i = tid; i < groups * 4; i += tt) tf[i] = make_uint4(0, 0, 0, 0);
}

// Candidate of one in-edge (tail u, weight wt) of a pull round, or kInf:
// only tails on the frontier count (every other tail's value has already
// been carried along all its out-edges), SSSP adds the weight and drops a
// sum at or above INF.
template <int A>
__device__ __forceinline__ int pull_cand(const Round& R, const unsigned char* vf, int u, int wt,
                                         Acc& acc) {
    if (!vf[u]) return kInf;
    acc.d++;
    const int x = R.val[u];
    if (A == SSSP) {
        const unsigned c = (unsigned)x + (unsigned)wt;
        return c < (unsigned)kInf ? (int)c : kInf;
    }
    return x;
}

// Pull round (the DSL's innbrs iterator, Sec. 2): every vertex v takes the
// least candidate over its in-edges -- SSSP: dist[u] + w over the weighted
// in-edge CSR; CC: label[u] over the both-directions rows -- from the tails
// on the current frontier, and lowers its own value with a plain store (no
// other lane writes v in this round).  Rows longer than the heavy threshold
// are served chunk by chunk, one atomic minimum per chunk.  Every vertex
// whose value drops goes on the next frontier with its out-row length
// counted; the frontier generation read here is cleared by the round's
// companion kernel once every wavefront has read it.  Values only decrease,
// so reading a tail that another wavefront lowers meanwhile is safe: the
// lowered tail is pushed and carried along its edges later.
template <int A>
__device__ void pull_round(const Round& R, Acc& acc) {
    const DevGraph& g = R.g;
    const int* irow = A == SSSP ? g.trow : g.srow;
    const int* icol = A == SSSP ? g.tcol : g.scol;
    const int* iw = A == SSSP ? g.tw : nullptr;
    const int2* ich = A == SSSP ? g.tchunks : g.shchunks;
    const long long nch = A == SSSP ? g.n_tchunks : g.n_shchunks;
    const int* orow = A == SSSP ? g.row : g.srow;
    const int n = g.n;
    const int cur = R.r & 1, nxt = cur ^ 1;
    const unsigned char* vf = R.ws.vflag[cur];
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const long long ntiles = (n + 63) / 64;
    __shared__ int s_pmin[4][64];  // blocks of 256 threads: four wavefronts
    int* smin = s_pmin[threadIdx.x >> 6];
    auto lower = [&](int v, int x, int old) {
        // v dropped from old to x: count it and put it on the next frontier
        if (x < old) {
            acc.u++;
            push(R, nxt, v);
            acc.p++;
            acc.add_f(orow[v + 1] - orow[v]);
        }
    };
    for (long long t = gw; t < ntiles; t += tw) {
        const int v = (int)(t * 64 + lane);
        int rb = 0, deg = 0;
        if (v < n) {
            rb = irow[v];
            deg = irow[v + 1] - rb;
            acc.v++;
        }
        const bool light = deg <= g.heavy;
        smin[lane] = kInf;
        __builtin_amdgcn_wave_barrier();
        // the in-edges of the tile's light rows, 64 per step, with the loads
        // of kBatch steps in flight: columns (and weights), then flags and
        // tail values; the minimum per row collects in LDS
        const int d = light ? deg : 0;
        const int incl = wave_incl_scan(d);
        const int total = __shfl(incl, 63, 64);
        const int excl = incl - d;
        for (int base = 0; base < total; base += 64 * kBatch) {
            int e[kBatch], slot[kBatch], u[kBatch], wt[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const int k = base + j * 64 + lane;
                int o = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int cand = o + step;
                    if (__shfl(excl, cand, 64) <= k) o = cand;
                }
                // every lane takes part in the shuffles (a lane past the end
                // still serves as a source for the others)
                const int eb = __shfl(rb, o, 64) + (k - __shfl(excl, o, 64));
                e[j] = k < total ? eb : -1;
                slot[j] = o;
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                u[j] = e[j] >= 0 ? icol[e[j]] : 0;
                wt[j] = (A == SSSP && e[j] >= 0) ? iw[e[j]] : 0;
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                if (e[j] < 0) continue;
                const int x = pull_cand<A>(R, vf, u[j], wt[j], acc);
                if (x < kInf) atomicMin(&smin[slot[j]], x);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (v < n && light) {
            acc.e += deg;
            const int x = smin[lane];
            const int old = R.val[v];
            if (x < old) R.val[v] = x;
            lower(v, x, old);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // heavy rows, one chunk per wavefront step: kBatch edges per lane
    for (long long k = gw; k < nch; k += tw) {
        const int2 c = ich[k];
        const int e1 = min(c.y + kChunk, irow[c.x + 1]);
        int u[kChunk / 64], wt[kChunk / 64];
#pragma unroll
        for (int j = 0; j < kChunk / 64; ++j) {
            const int e = c.y + j * 64 + lane;
            u[j] = e < e1 ? icol[e] : -1;
            wt[j] = (A == SSSP && e < e1) ? iw[e] : 0;
        }
        int x = kInf;
#pragma unroll
        for (int j = 0; j < kChunk / 64; ++j)
            if (u[j] >= 0) x = min(x, pull_cand<A>(R, vf, u[j], wt[j], acc));
#pragma unroll
        for (int dd = 32; dd > 0; dd >>= 1) x = min(x, __shfl_xor(x, dd, 64));
        if (lane == 0) {
            acc.e += e1 - c.y;
            if (x < kInf) lower(c.x, x, atomicMin(&R.val[c.x], x));
        }
    }
}

// SSSP with a per-round choice between pushing the frontier (the worklist
// round of Sec. 3.3, heavy out-rows to the chunk kernel) and pulling every
// vertex over its in-edges (the innbrs iterator) when the frontier's
// out-edges are a large part of the graph: a pull round needs no atomics on
// light rows and reads each in-edge's tail flag before its value.
__global__ __launch_bounds__(256) void k_sssp_diropt(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    Ctl* ctl = R.ws.ctl;
    const bool pull = R.r > 0 && prev_front(R) * kSsspPullRatio > (long long)R.g.m;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->pull[R.r % 3] = pull;
        ctl->hgrid[R.r % 3] = 0;  // rewritten by this round's heavy kernel
    }
    Acc acc;
    if (pull)
        pull_round<SSSP>(R, acc);
    else
        vasync_body<SSSP, MAP_BALANCED>(R, acc, false, kInf);
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Heavy rows of the frontier: the light kernel of the same round marked
// them in the round's bitmap; every wavefront walks the static chunk list
// and serves the chunks whose row is marked.
template <int A>
__global__ __launch_bounds__(256) void k_heavy(Round R) {
    Ctl* ctl = R.ws.ctl;
    if (*(volatile int*)&ctl->done) return;
    const DevGraph& g = R.g;
    const int* row = A == CC ? g.srow : g.row;
    const int* col = A == CC ? g.scol : g.col;
    const int2* chunks = A == CC ? g.shchunks : g.hchunks;
    const long long nch = A == CC ? g.n_shchunks : g.n_hchunks;
    const int nxt = (R.r & 1) ^ 1;
    const int wpb = blockDim.x >> 6;
    const long long gw = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
    const long long tw = (long long)gridDim.x * wpb;
    const int lane = threadIdx.x & 63;
    const bool nf = A == SSSP && R.delta > 0;
    const int bound = nf ? *(volatile int*)&ctl->bound[R.r % 3] : kInf;
    // a pulling BFS round or a sweeping CC round marks no heavy row:
    // nothing to serve
    const bool pulled = (A == BFS || ((A == CC || A == SSSP) && R.fedges)) &&
                        *(volatile int*)&ctl->pull[R.r % 3] != 0;
    Acc acc;
    // an SSSP pull round read the frontier generation without consuming it:
    // it is cleared here, once the round kernel has completed
    if (A == SSSP && pulled) clear_generation(R, R.r & 1);
    // 64 chunks' rows are checked at once, then the wavefront serves the
    // chunks that match.  The 64 chunks of one check are spread over the
    // list with the stride of the whole grid, so that the chunks of one long
    // row (which sit next to each other) land on different wavefronts, and
    // every wavefront gets a like mix of long and short rows.  (Checking 64
    // consecutive entries instead, with the list ordered so that a row's
    // chunks lie far apart, loads the descriptors coalesced but gave the
    // first wavefronts the hubs' full chunks: rmat22 79.4 -> 75.3 GTEPS.)
    for (long long k0 = 0; !pulled && gw + k0 * tw < nch; k0 += 64) {
        const long long it = gw + (k0 + lane) * tw;
        int2 c = make_int2(0, 0);
        bool on = false;
        if (it < nch) {
            c = chunks[it];
            on = heavy_marked(R, c.x);
        }
        // each lane fetches its own matched chunk's end now, all in
        // parallel, instead of one chunk at a time below.  The tail value is
        // read when the chunk is served: read here it would miss the
        // decreases that other wavefronts make meanwhile (measured: weaker
        // relaxations, more rounds).  BFS: the round's level, or under local
        // expansion (levels differ within a round) the row's own level,
        // lowered atomically.
        const bool lvl = A == BFS && R.hops == 0;
        const int cend = on ? min(c.y + kChunk, row[c.x + 1]) : 0;
        unsigned long long am = __ballot(on);
        while (am) {
            const int o = __ffsll(am) - 1;
            am &= am - 1;
            const int e0 = __shfl(c.y, o, 64), e1 = __shfl(cend, o, 64);
            const int sv = lvl ? R.r : R.val[__shfl(c.x, o, 64)];
            if (A == BFS && !lvl)
                wave_relax_range<A, true, batch_for(A, false), true>(R, col, e0, e1, sv, nxt, acc,
                                                                     bound);
            else
                wave_relax_range<A, true, batch_for(A, false)>(R, col, e0, e1, sv, nxt, acc, bound);
        }
    }
    if (nf) nearfar_finish(R, acc);
    block_finish(R, acc, R.r % 3, KIND_HEAVY);
}

// CC shortcut pass used after an edge sweep: label[v] = label[label[v]].
// Under the per-round schedule it runs after sweeping rounds only, puts the
// vertices it lowers on the next frontier, and records that frontier in the
// heavy kernel's push-count row (the heavy kernel idles in those rounds).
__global__ __launch_bounds__(256) void k_jump(Round R) {
    const Ctl* ctl = R.ws.ctl;
    if (*(volatile const int*)&ctl->done) return;
    if (R.fedges && *(volatile const int*)&ctl->pull[R.r % 3] == 0) return;
    const int n = R.g.n;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    Acc acc;
    // a pulling round read its frontier generation without consuming it
    if (R.pullmode) clear_generation(R, R.r & 1);
    for (long long v = R.jump ? tid : n; v < n; v += tt) {
        const int x = R.val[v];
        const int y = R.val[x];
        if (y < x) {
            const int old = atomicMin(&R.val[v], y);
            if (y < old) {
                acc.u++;
                if (R.fedges) sweep_push(R, (int)v, acc);
            }
        }
    }
    block_finish(R, acc, R.r % 3, KIND_AUX, R.fedges ? KIND_HEAVY : -1);
}

// CC with a per-round choice between the two schedules of the paper (a
// topology-driven sweep, Algorithm 2's edge form, and the data-driven
// worklist of Sec. 3.3).  Round r sweeps every stored edge while the rows of
// the frontier left by round r-1 hold more than 1/kSweepRatio of the
// both-directions edges (always in round 0), else it serves that frontier
// from the both-directions CSR.  A sweep puts every vertex it lowers on the
// next frontier (so a later worklist round sees every vertex whose value
// changed after its edges were last read) and clears the frontier it skips.
__global__ __launch_bounds__(256) void k_cc_diropt(Round R) {
    if (!round_begin(R)) return;
    clear_prev_heavy(R);
    Ctl* ctl = R.ws.ctl;
    const long long front = R.r > 0 ? prev_front(R) : (long long)R.g.ms;
    const bool sweep = front * kSweepRatio > (long long)R.g.ms || R.r == 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->pull[R.r % 3] = sweep;
        ctl->hgrid[R.r % 3] = 0;  // rewritten by this round's heavy or shortcut kernel
    }
    Acc acc;
    if (sweep && R.pullmode && R.r > 0) {
        // vertex-based dense round: every vertex pulls the labels of its
        // frontier neighbours (the shortcut kernel clears the generation)
        pull_round<CC>(R, acc);
    } else if (sweep) {
        // the frontier generation of this round is not read: clear it
        clear_generation(R, R.r & 1);
        if (R.r == 0) {
            cc_first_pass(R, acc);
        } else {
            esync_body<CC, true>(R, acc);
            acc.d = acc.e;
        }
    } else {
        vasync_body<CC, MAP_BALANCED>(R, acc, false, kInf);
    }
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// ------------------------------------------------------- graph build ----

// Edge-list sources: src[e] = the row u with row[u] <= e < row[u+1].  A
// block takes kFillWin consecutive edges.  The row of the window's first edge
// comes from a binary search of row[]; every row that starts inside the
// window writes its number at its first edge (in LDS); a running maximum over
// the window then carries each row number to the rest of its edges.  The
// work per window is the same whatever the degrees are.
constexpr int kFillWin = 4096;
__device__ __forceinline__ int fill_slot(int i) { return i + (i >> 4); }  // 16 + 1 padding

__device__ __forceinline__ int row_of_edge(const int* row, int n, long long e) {
    // invariant row[lo] <= e < row[hi]; row[0] = 0 and row[n] = m > e
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = lo + ((hi - lo) >> 1);
        if (row[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_fill_src(const int* row, int n, int m, int* src) {
    constexpr int PT = kFillWin / 256;
    __shared__ int s_row[kFillWin + kFillWin / 16];
    __shared__ int s_r[2];
    __shared__ int s_wmax[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (long long wb = blockIdx.x; wb * kFillWin < m; wb += gridDim.x) {
        const long long e0 = wb * kFillWin;
        const int len = (int)min((long long)kFillWin, (long long)m - e0);
        if (threadIdx.x < 2) s_r[threadIdx.x] = row_of_edge(row, n, threadIdx.x ? e0 + len - 1 : e0);
        for (int i = threadIdx.x; i < kFillWin; i += 256) s_row[fill_slot(i)] = -1;
        __syncthreads();
        const int r0 = s_r[0], r1 = s_r[1];
        // rows r0+1..r1 start inside the window, after its first edge
        for (long long u = (long long)r0 + 1 + threadIdx.x; u <= r1; u += 256) {
            const int b = row[u];
            if (row[u + 1] > b) s_row[fill_slot((int)(b - e0))] = (int)u;
        }
        __syncthreads();
        // thread t owns entries [t*PT, t*PT + PT): block-wide exclusive
        // maximum of the per-thread maxima, then the running maximum
        int mx = -1;
#pragma unroll
        for (int j = 0; j < PT; ++j) mx = max(mx, s_row[fill_slot(threadIdx.x * PT + j)]);
        int x = mx;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (lane >= d) x = max(x, y);
        }
        if (lane == 63) s_wmax[wid] = x;
        __syncthreads();
        int c = r0;
        for (int i = 0; i < wid; ++i) c = max(c, s_wmax[i]);
        const int before = __shfl_up(x, 1, 64);
        if (lane > 0) c = max(c, before);
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int k = fill_slot(threadIdx.x * PT + j);
            c = max(c, s_row[k]);
            s_row[k] = c;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += 256) src[e0 + i] = s_row[fill_slot(i)];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_count_in(const int* col, int m, int* indeg) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long e = tid; e < m; e += tt) atomicAdd(&indeg[col[e]], 1);
}

// Both-directions CSR: row u holds u's out-edges (input order) followed by
// the tails of its in-edges (order unspecified).
__global__ __launch_bounds__(256) void k_sym_fill(const int* row, const int* col, const int* src,
                                                  int m, const int* srow, int* cursor, int* scol) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long e = tid; e < m; e += tt) {
        const int u = src[e], v = col[e];
        scol[srow[u] + (int)(e - row[u])] = v;
        const int pos = srow[v] + (row[v + 1] - row[v]) + atomicAdd(&cursor[v], 1);
        scol[pos] = u;
    }
}

// Upload checks of the edge arrays: the smallest and largest column, the
// smallest and largest weight (stats[0..3]) and the weight sum.  One atomic
// per block and statistic.
__global__ __launch_bounds__(256) void k_check(const int* col, const int* w, int m, int* stats,
                                               unsigned long long* wsum) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    int cmin = 2147483647, cmax = -2147483647 - 1, wmin = 2147483647, wmax = -2147483647 - 1;
    unsigned long long sum = 0;
    for (long long e = tid; e < m; e += tt) {
        const int c = col[e];
        cmin = min(cmin, c);
        cmax = max(cmax, c);
        if (w) {
            const int x = w[e];
            wmin = min(wmin, x);
            wmax = max(wmax, x);
            sum += (unsigned long long)(long long)x;  // the total's sign is checked by wmin
        }
    }
    __shared__ int s4[4][4];
    __shared__ unsigned long long ss[4];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        cmin = min(cmin, __shfl_xor(cmin, d, 64));
        cmax = max(cmax, __shfl_xor(cmax, d, 64));
        wmin = min(wmin, __shfl_xor(wmin, d, 64));
        wmax = max(wmax, __shfl_xor(wmax, d, 64));
        sum += __shfl_xor(sum, d, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s4[wid][0] = cmin;
        s4[wid][1] = cmax;
        s4[wid][2] = wmin;
        s4[wid][3] = wmax;
        ss[wid] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            cmin = min(cmin, s4[i][0]);
            cmax = max(cmax, s4[i][1]);
            wmin = min(wmin, s4[i][2]);
            wmax = max(wmax, s4[i][3]);
            sum += ss[i];
        }
        atomicMin(&stats[0], cmin);
        atomicMax(&stats[1], cmax);
        atomicMin(&stats[2], wmin);
        atomicMax(&stats[3], wmax);
        atomicAdd(wsum, sum);
    }
}

// Stable split of the edge list by the part of each edge's head (part[v] in
// [0, kXcd)), CSR order kept inside a part.  Block b owns edges
// [b * kSplitTile, (b + 1) * kSplitTile): the first kernel counts its edges
// per part, the second places them at base[b][p] onwards, 256 edges at a
// time, ranked by ballots so that the order is kept.
constexpr int kSplitTile = 4096;

__global__ __launch_bounds__(256) void k_split_count(const int* col, int m,
                                                     const unsigned char* part, int* counts) {
    __shared__ int c[kXcd];
    if (threadIdx.x < kXcd) c[threadIdx.x] = 0;
    __syncthreads();
    const long long e0 = (long long)blockIdx.x * kSplitTile;
    const long long e1 = min(e0 + kSplitTile, (long long)m);
    for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&c[part[col[e]]], 1);
    __syncthreads();
    if (threadIdx.x < kXcd) counts[(long long)blockIdx.x * kXcd + threadIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_split_place(const int* src, const int* col, const int* w,
                                                     int m, const unsigned char* part,
                                                     const long long* base, int* psrc, int* pcol,
                                                     int* pw) {
    __shared__ long long off[kXcd];
    __shared__ int wc[4][kXcd];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x < kXcd) off[threadIdx.x] = base[(long long)blockIdx.x * kXcd + threadIdx.x];
    __syncthreads();
    const long long e0 = (long long)blockIdx.x * kSplitTile;
    const long long e1 = min(e0 + kSplitTile, (long long)m);
    for (long long t = e0; t < e1; t += blockDim.x) {
        const long long e = t + threadIdx.x;
        int p = -1, u = 0, v = 0, x = 0;
        if (e < e1) {
            u = src[e];
            v = col[e];
            if (w) x = w[e];
            p = part[v];
        }
        long long at = -1;
        for (int q = 0; q < kXcd; ++q) {
            const unsigned long long mk = __ballot(p == q);
            if (lane == 0) wc[wid][q] = __popcll(mk);
            if (p == q) at = __popcll(mk & ((1ull << lane) - 1));
        }
        __syncthreads();
        if (p >= 0) {
            long long o = off[p] + at;
            for (int i = 0; i < wid; ++i) o += wc[i][p];
            psrc[o] = u;
            pcol[o] = v;
            if (w) pw[o] = x;
        }
        __syncthreads();
        if (threadIdx.x < kXcd) {
            int tot = 0;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += wc[i][threadIdx.x];
            off[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

// In-edge CSR with weights: the tails and weights of v's in-edges at
// trow[v] + (a slot claimed with a counter; the order inside a row is
// unspecified).
__global__ __launch_bounds__(256) void k_t_fill(const int* col, const int* w, const int* src,
                                                int m, const int* trow, int* cursor, int* tcol,
                                                int* tw) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long e = tid; e < m; e += tt) {
        const int v = col[e];
        const int pos = trow[v] + atomicAdd(&cursor[v], 1);
        tcol[pos] = src[e];
        tw[pos] = w ? w[e] : 1;
    }
}

// ----------------------------------------------------- CC by union-find ----
// The DSL's Set type is a union-find structure (Sec. 2); CC over it, in the
// order of Sutton, Ben-Nun and Barak's Afforest: every vertex is linked with
// its first neighbour (phase 0) and its second (phase 1) in the
// both-directions rows, each followed by a compression; phase 2 samples the
// roots of 1024 vertices and takes the most frequent as the giant
// component's; phase 3 links, for every vertex outside that component, all
// its remaining neighbours (an edge with one end in the giant component is
// seen from the other end; edges inside it need nothing), and a last
// compression makes every parent a root.  Linking hangs the larger of two
// roots under the smaller with a compare-and-swap, so a root is always the
// smallest id of its tree, and the parent array ends as the smallest id of
// each component -- the labels of the other schedules.  The value array is
// the parent array (labels start as the ids).  Phases set the round's
// change flag except the last, so the round after it ends the traversal.
__device__ __forceinline__ int uf_load(int* p, int x) {
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x while other lanes link: path halving (only non-roots change).
__device__ __forceinline__ int uf_find(int* parent, int x) {
    int p = uf_load(parent, x);
    while (p != x) {
        const int gp = uf_load(parent, p);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
        p = uf_load(parent, x);
    }
    return x;
}

__device__ __forceinline__ bool uf_link(int* parent, int a, int b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return false;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expect = a;  // a > b: hang root a under root b
        if (__hip_atomic_compare_exchange_strong(parent + a, &expect, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return true;
    }
}

__global__ __launch_bounds__(256) void k_uf(Round R) {
    if (!round_begin(R)) return;
    const DevGraph& g = R.g;
    int* parent = R.val;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    Acc acc;
    if (R.r <= 1) {
        for (long long v = tid; v < g.n; v += tt) {
            const int b = g.srow[v];
            if (g.srow[v + 1] - b > R.r) {
                acc.e++;
                acc.u += uf_link(parent, (int)v, g.scol[b + R.r]);
            }
        }
    } else if (R.r == 2) {
        // the giant component's root: the most frequent root of 1024
        // vertices spread over the ids (a multiplicative hash of i)
        __shared__ int s_root[1024];
        if (blockIdx.x == 0) {
            for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
                const unsigned h = (unsigned)i * 2654435761u;
                s_root[i] = parent[(int)((unsigned long long)h * (unsigned)g.n >> 32)];
            }
            __syncthreads();
            int best = -1, best_count = 0;
            for (int i = threadIdx.x; i < 1024; i += blockDim.x) {
                int c = 0;
                for (int k = 0; k < 1024; ++k) c += s_root[k] == s_root[i];
                if (c > best_count || (c == best_count && s_root[i] < best)) {
                    best_count = c;
                    best = s_root[i];
                }
            }
            __shared__ int s_bc[256], s_b[256];
            s_bc[threadIdx.x] = best_count;
            s_b[threadIdx.x] = best;
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int i = 1; i < (int)blockDim.x; ++i)
                    if (s_bc[i] > best_count || (s_bc[i] == best_count && s_b[i] < best)) {
                        best_count = s_bc[i];
                        best = s_b[i];
                    }
                R.ws.ctl->giant = best;
            }
        }
    } else if (R.r == 3) {
        const int giant = *(volatile int*)&R.ws.ctl->giant;
        for (long long v = tid; v < g.n; v += tt) {
            if (parent[v] == giant) continue;  // roots after the compression
            const int b = g.srow[v], e1 = g.srow[v + 1];
            for (int e = b + 2; e < e1; ++e) {
                acc.e++;
                acc.u += uf_link(parent, (int)v, g.scol[e]);
            }
        }
    }
    // phases 0-2 keep the traversal going (one push on the books); the
    // last one changes nothing the next round would read
    if (R.r < 3) acc.p = tid == 0;
    else acc.u = acc.p = 0;
    block_finish(R, acc, R.r % 3, KIND_ROUND);
}

// Every parent to its root; each thread writes its own vertex only.
__global__ __launch_bounds__(256) void k_uf_compress(Round R) {
    if (*(volatile int*)&R.ws.ctl->done) return;
    int* parent = R.val;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < R.g.n; v += tt) {
        int x = parent[v];
        while (parent[x] != x) x = parent[x];
        parent[v] = x;
    }
}

// ------------------------------------------------------- renumbering ----
// A graph stored with its vertices renumbered (new id newid[v] for caller id
// v, oldid[] the inverse) keeps each row's edges in order: caller edge e of
// row u lands at nrow[newid[u]] + (e - row[u]).

__global__ __launch_bounds__(256) void k_renumber(const int* row, const int* col, const int* w,
                                                  const int* src, int m, const int* newid,
                                                  const int* nrow, int* ncol, int* nw,
                                                  int* eorig, int* epos) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long e = tid; e < m; e += tt) {
        const int u = src[e];
        const int p = nrow[newid[u]] + (int)(e - row[u]);
        ncol[p] = newid[col[e]];
        if (nw) nw[p] = w[e];
        if (eorig) eorig[p] = (int)e;
        if (epos) epos[e] = p;
    }
}

// Output in the caller's order: a coalesced read of newid, one gather (none
// for a vertex without edges: it is reached only as the source).
__global__ __launch_bounds__(256) void k_unrenumber(int* out, const int* val, const int* newid,
                                                    int n, int n_active, int source) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < n; v += tt) {
        const int k = newid[v];
        out[v] = k < n_active ? val[k] : (v == source ? 0 : kInf);
    }
}

// CC on a renumbered graph: the label of a component is the least of the
// caller's ids among its vertices, while the propagation left the least new
// id.  Each block takes a contiguous range of new ids and keeps, per lane, a
// running (label, least caller id) pair, written out with a checked atomic
// minimum whenever the label changes; hottest-first numbering puts most of
// the large components' vertices next to each other, so the pairs change
// rarely.  The last pairs are merged per wavefront and per block before
// their atomics, which keeps the atomics on one label (the giant component)
// to about one per block.
__global__ __launch_bounds__(256) void k_cc_min_ids(const int* label, const int* oldid, int* rmin,
                                                    int n) {
    const long long per = ((long long)n + gridDim.x - 1) / gridDim.x;
    const long long v0 = (long long)blockIdx.x * per;
    const long long v1 = min((long long)n, v0 + per);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int L = -1, mn = kInf;
    for (long long v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        const int l = label[v];
        const int o = oldid[v];
        if (l != L) {
            if (L >= 0 && mn < rmin[L]) atomicMin(&rmin[L], mn);
            L = l;
            mn = o;
        } else {
            mn = min(mn, o);
        }
    }
    // wavefront: the lanes sharing the first active lane's label reduce
    const unsigned long long act = __ballot(L >= 0);
    int wl = -1, wm = kInf;
    if (act) {
        const int leader = __ffsll(act) - 1;
        wl = __shfl(L, leader, 64);
        const bool same = L == wl;
        int x = same ? mn : kInf;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) x = min(x, __shfl_xor(x, d, 64));
        wm = x;
        if (!same && L >= 0 && mn < rmin[L]) atomicMin(&rmin[L], mn);
    }
    // block: the wavefronts' pairs, merged by label
    __shared__ int s_l[4], s_m[4];
    if (lane == 0) {
        s_l[wid] = wl;
        s_m[wid] = wm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (int)(blockDim.x >> 6);
        for (int i = 0; i < nw; ++i) {
            if (s_l[i] < 0) continue;
            int x = s_m[i];
            for (int j = i + 1; j < nw; ++j)
                if (s_l[j] == s_l[i]) {
                    x = min(x, s_m[j]);
                    s_l[j] = -1;
                }
            if (x < rmin[s_l[i]]) atomicMin(&rmin[s_l[i]], x);
        }
    }
}

__global__ __launch_bounds__(256) void k_cc_min_out(int* out, const int* label, const int* newid,
                                                    const int* rmin, int n, int n_active) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < n; v += tt) {
        const int k = newid[v];
        out[v] = k < n_active ? rmin[label[k]] : (int)v;
    }
}

// ----------------------------------------------------- launch wrappers ----

// Blocks of `block` threads of kernel f that fit on the device at once.  A
// grid-stride kernel launched with more blocks than this would run its last
// blocks in a second wave, so every launch is clamped to it.
static int resident_cap(const void* f, int block) {
    int occ = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1 << 30;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1 << 30;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, block, 0) != hipSuccess || occ < 1)
        return 1 << 30;
    return occ * cus;
}

#define GG_LAUNCH(kernel, grid, block, s, ...)                                       \
    do {                                                                             \
        static const int cap_ = resident_cap(reinterpret_cast<const void*>(kernel), (block)); \
        const int g_ = (grid) < cap_ ? (grid) : cap_;                                \
        hipLaunchKernelGGL(kernel, dim3(g_), dim3(block), 0, s, __VA_ARGS__);        \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_init(const Round& R, int algo, bool async, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_init, grid, block, s, R, algo, async ? 1 : 0);
}

hipError_t launch_seed(const Round& R, bool async, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_seed, grid, block, s, R, async ? 1 : 0);
}

template <int A>
static hipError_t vsync_a(const Round& R, int grid, int block, hipStream_t s) {
    switch (R.mapping) {
        case MAP_THREAD: GG_LAUNCH((k_vsync<A, MAP_THREAD>), grid, block, s, R);
        case MAP_WAVE: GG_LAUNCH((k_vsync<A, MAP_WAVE>), grid, block, s, R);
        default: GG_LAUNCH((k_vsync<A, MAP_BALANCED>), grid, block, s, R);
    }
}

hipError_t launch_vsync(const Round& R, int algo, int grid, int block, hipStream_t s) {
    switch (algo) {
        case SSSP: return vsync_a<SSSP>(R, grid, block, s);
        case BFS: return vsync_a<BFS>(R, grid, block, s);
        default: return vsync_a<CC>(R, grid, block, s);
    }
}

hipError_t launch_esync(const Round& R, int algo, int grid, int block, hipStream_t s) {
    switch (algo) {
        case SSSP: GG_LAUNCH(k_esync<SSSP>, grid, block, s, R);
        case BFS: GG_LAUNCH(k_esync<BFS>, grid, block, s, R);
        default: GG_LAUNCH(k_esync<CC>, grid, block, s, R);
    }
}

// Resident blocks per CU for the local-expansion round kernels.  Their
// rounds wait for the slowest wavefront, and a CU holding a seventh block
// slows its wavefronts: grid4096 BFS (the BFS form fits seven blocks per CU)
// took 50 us per round with 1,792 blocks, 46 us with 1,600 and 39 us with
// 1,536 or fewer.
constexpr int kLocalBlocksPerCu = 6;

static int local_grid(int grid) {
    static const int cap = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            return 1 << 30;
        return kLocalBlocksPerCu * cus;
    }();
    return grid < cap ? grid : cap;
}

template <int A>
static hipError_t vasync_a(const Round& R, int grid, int block, hipStream_t s) {
    switch (R.mapping) {
        case MAP_THREAD: GG_LAUNCH((k_vasync<A, MAP_THREAD>), grid, block, s, R);
        case MAP_WAVE: GG_LAUNCH((k_vasync<A, MAP_WAVE>), grid, block, s, R);
        default:
            if constexpr (A == SSSP)
                if (R.delta > 0) {
                    if (R.hops > 0) GG_LAUNCH((k_vlocal<A, true>), local_grid(grid), block, s, R);
                    GG_LAUNCH((k_vasync<A, MAP_BALANCED, true>), grid, block, s, R);
                }
            if (R.hops > 0) GG_LAUNCH((k_vlocal<A, false>), local_grid(grid), block, s, R);
            GG_LAUNCH((k_vasync<A, MAP_BALANCED>), grid, block, s, R);
    }
}

hipError_t launch_vasync(const Round& R, int algo, int grid, int block, hipStream_t s) {
    switch (algo) {
        case SSSP: return vasync_a<SSSP>(R, grid, block, s);
        case BFS: return vasync_a<BFS>(R, grid, block, s);
        default: return vasync_a<CC>(R, grid, block, s);
    }
}

hipError_t launch_easync(const Round& R, int algo, int grid, int block, hipStream_t s) {
    switch (algo) {
        case SSSP: GG_LAUNCH(k_easync<SSSP>, grid, block, s, R);
        case BFS: GG_LAUNCH(k_easync<BFS>, grid, block, s, R);
        default: GG_LAUNCH(k_easync<CC>, grid, block, s, R);
    }
}

hipError_t launch_heavy(const Round& R, int algo, int grid, int block, hipStream_t s) {
    switch (algo) {
        case SSSP: GG_LAUNCH(k_heavy<SSSP>, grid, block, s, R);
        case BFS: GG_LAUNCH(k_heavy<BFS>, grid, block, s, R);
        default: GG_LAUNCH(k_heavy<CC>, grid, block, s, R);
    }
}

hipError_t launch_bfs_diropt(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_bfs_diropt, grid, block, s, R);
}

hipError_t launch_cc_diropt(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_cc_diropt, grid, block, s, R);
}

hipError_t launch_sssp_diropt(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_sssp_diropt, grid, block, s, R);
}

__global__ __launch_bounds__(64) void k_mark(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_uf(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_uf, grid, block, s, R);
}

hipError_t launch_uf_compress(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_uf_compress, grid, block, s, R);
}

hipError_t launch_mark(unsigned long long* p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_mark, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_jump(const Round& R, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_jump, grid, block, s, R);
}

hipError_t launch_fill_src(const int* row, int n, int m, int* src, int grid, int block,
                           hipStream_t s) {
    GG_LAUNCH(k_fill_src, grid, block, s, row, n, m, src);
}

hipError_t launch_count_in(const int* col, int m, int* indeg, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_count_in, grid, block, s, col, m, indeg);
}

hipError_t launch_sym_fill(const int* row, const int* col, const int* src, int n, int m,
                           const int* srow, int* cursor, int* scol, int grid, int block,
                           hipStream_t s) {
    (void)n;
    GG_LAUNCH(k_sym_fill, grid, block, s, row, col, src, m, srow, cursor, scol);
}

hipError_t launch_t_fill(const int* col, const int* w, const int* src, int m, const int* trow,
                         int* cursor, int* tcol, int* tw, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_t_fill, grid, block, s, col, w, src, m, trow, cursor, tcol, tw);
}

hipError_t launch_check(const int* col, const int* w, int m, int* stats,
                        unsigned long long* wsum, int grid, hipStream_t s) {
    GG_LAUNCH(k_check, grid, 256, s, col, w, m, stats, wsum);
}

int split_blocks(long long m) { return (int)((m + kSplitTile - 1) / kSplitTile); }

hipError_t launch_renumber(const int* row, const int* col, const int* w, const int* src, int m,
                           const int* newid, const int* nrow, int* ncol, int* nw, int* eorig,
                           int* epos, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_renumber, grid, block, s, row, col, w, src, m, newid, nrow, ncol, nw, eorig, epos);
}

hipError_t launch_unrenumber(int* out, const int* val, const int* newid, int n, int n_active,
                             int source, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_unrenumber, grid, block, s, out, val, newid, n, n_active, source);
}

hipError_t launch_cc_min_ids(const int* label, const int* oldid, int* rmin, int n, int grid,
                             int block, hipStream_t s) {
    // one contiguous range per block (the block-level merge assumes 4 waves)
    if (block != 256) return hipErrorInvalidValue;
    GG_LAUNCH(k_cc_min_ids, grid, block, s, label, oldid, rmin, n);
}

hipError_t launch_cc_min_out(int* out, const int* label, const int* newid, const int* rmin,
                             int n, int n_active, int grid, int block, hipStream_t s) {
    GG_LAUNCH(k_cc_min_out, grid, block, s, out, label, newid, rmin, n, n_active);
}

hipError_t launch_split_count(const int* col, int m, const unsigned char* part, int* counts,
                              hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_count, dim3(split_blocks(m)), dim3(256), 0, s, col, m, part,
                       counts);
    return hipGetLastError();
}

hipError_t launch_split_place(const int* src, const int* col, const int* w, int m,
                              const unsigned char* part, const long long* base, int* psrc,
                              int* pcol, int* pw, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_place, dim3(split_blocks(m)), dim3(256), 0, s, src, col, w, m,
                       part, base, psrc, pcol, pw);
    return hipGetLastError();
}

}  // namespace gg
