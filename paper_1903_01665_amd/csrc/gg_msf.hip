// gg_msf.hip -- minimum spanning forest on the device (gg_msf in include/gg.h).
//
// MST is the fourth algorithm of the paper's evaluation (Sec. 4.1, Table 3);
// the DSL's Set type is a union-find structure (Sec. 2).  Every stored edge
// e = (src[e], col[e]) with weight w[e] is an undirected edge with the key
// w[e] * 2^32 + e: keys are distinct, so the forest of least keys is unique
// and every run returns the same edge set.  On a renumbered graph e is the
// caller's index of the edge (eorig of its stored place; epos maps back), so
// keys, ties and the output flags are those of the caller's edge order.
//
// Boruvka rounds, four kernels each:
//   min      every edge whose ends lie in different components offers its key
//            to both components (64-bit atomic minimum, checked first with a
//            plain load); a component is named by its union-find root, and
//            between rounds every vertex points at its root
//   link     every component with an offer joins the forest with its least
//            edge (cut property) and merges with the other end's component
//            in a lock-free union-find: the larger root is linked under the
//            smaller one by compare-and-swap, so links never form a cycle;
//            two components that chose the same edge mark it once
//   compress, every vertex points at its root again: a pass with path
//   settle   halving shortens the trees, then a pass in which every thread
//            writes only its own vertex (a halving store of the first pass
//            can land after the owner's own store, leaving an ancestor that
//            is not the root; the offers of the next round need the root)
// A round with no crossing edge ends the run; the next round's first kernel
// reports it (same protocol as the traversal rounds).  Each round at least
// halves the number of components that still have a crossing edge, so
// log2(n) + 2 rounds suffice.

#include <new>

#include "gg_runtime.h"

using namespace gg;

namespace {

constexpr unsigned long long kNoEdge = ~0ull;
constexpr int kMsfMaxRounds = 40;
constexpr int kMsfBatch = 4;

struct Msf {
    const int* src;
    const int* col;
    const int* w;
    const int* eorig;          // renumbered graph: caller's index of each stored edge
    const int* epos;           // ... and stored place of each caller edge (else null)
    int n, m;
    int* parent;               // union-find forest
    unsigned long long* best;  // per root: least key of a crossing edge
    unsigned char* in_msf;     // [m] output
    Ctl* ctl;
    Stat* stat;
    int* host_done;
    int tag;
    int r;
};

__device__ __forceinline__ int wsum(int x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Per-block plain update of a statistics slot (edges, updates) and of the
// round's flag.
__device__ void msf_finish(const Msf& M, int kind, int edges, int crossing, int links) {
    __shared__ int s_v[3][4];
    const int a = wsum(edges), b = wsum(crossing), c = wsum(links);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_v[0][wid] = a;
        s_v[1][wid] = b;
        s_v[2][wid] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long E = 0, X = 0, L = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            E += s_v[0][i];
            X += s_v[1][i];
            L += s_v[2][i];
        }
        if (E | X | L) {
            Stat* st = M.stat + kind * kMaxStatBlocks + blockIdx.x;
            st->edges += E;
            st->verts += X;
            st->updates += L;
        }
        if (X > 0) M.ctl->changed[M.r % 3] = 1;
    }
}

__global__ __launch_bounds__(256) void k_msf_init(Msf M) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < M.n; v += tt) {
        M.parent[v] = (int)v;
        M.best[v] = kNoEdge;
    }
    for (long long e = tid; e < M.m; e += tt) M.in_msf[e] = 0;
    for (long long i = tid; i < kKinds * kMaxStatBlocks; i += tt) M.stat[i] = Stat{0, 0, 0, 0, 0};
    if (tid == 0) *M.ctl = Ctl{};
}

// Round entry: false once the run has ended (the kernel that sees round r-1
// without a crossing edge records the round count and tells the host).
__device__ __forceinline__ bool msf_begin(const Msf& M) {
    Ctl* ctl = M.ctl;
    if (*(volatile int*)&ctl->done) return false;
    if (M.r > 0 && *(volatile int*)&ctl->changed[(M.r - 1) % 3] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->iters = M.r;
            ctl->done = 1;
            __hip_atomic_store(M.host_done, M.tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return false;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->changed[(M.r + 1) % 3] = 0;
    return true;
}

__device__ __forceinline__ bool offer(const Msf& M, int u, int v, int e) {
    if (u == v) return false;
    const int ru = M.parent[u], rv = M.parent[v];
    if (ru == rv) return false;
    const int eo = M.eorig ? M.eorig[e] : e;
    const unsigned long long key = ((unsigned long long)(unsigned)M.w[e] << 32) | (unsigned)eo;
    if (key < M.best[ru]) atomicMin(&M.best[ru], key);
    if (key < M.best[rv]) atomicMin(&M.best[rv], key);
    return true;
}

__global__ __launch_bounds__(256) void k_msf_min(Msf M) {
    if (!msf_begin(M)) return;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    int edges = 0, crossing = 0;
    const long long m4 = M.m & ~3LL;
    for (long long e = tid * 4; e < m4; e += tt * 4) {
        const int4 s4 = *reinterpret_cast<const int4*>(M.src + e);
        const int4 c4 = *reinterpret_cast<const int4*>(M.col + e);
        edges += 4;
        crossing += offer(M, s4.x, c4.x, (int)e);
        crossing += offer(M, s4.y, c4.y, (int)e + 1);
        crossing += offer(M, s4.z, c4.z, (int)e + 2);
        crossing += offer(M, s4.w, c4.w, (int)e + 3);
    }
    for (long long e = m4 + tid; e < M.m; e += tt) {
        edges++;
        crossing += offer(M, M.src[e], M.col[e], (int)e);
    }
    msf_finish(M, KIND_ROUND, edges, crossing, 0);
}

// Union-find accesses while links happen: device-scope atomics, so every
// die sees the links of the others.  Path halving only rewrites vertices
// that are no longer roots, which no link touches.
__device__ __forceinline__ int load_parent(int* p, int x) {
    return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_linking(int* parent, int x) {
    int p = load_parent(parent, x);
    while (p != x) {
        const int gp = load_parent(parent, p);
        if (gp != p)
            __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
        p = load_parent(parent, x);
    }
    return x;
}

__global__ __launch_bounds__(256) void k_msf_link(Msf M) {
    if (*(volatile int*)&M.ctl->done || *(volatile int*)&M.ctl->changed[M.r % 3] == 0) return;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    int links = 0;
    for (long long v = tid; v < M.n; v += tt) {
        const unsigned long long b = M.best[v];
        if (b == kNoEdge) continue;
        M.best[v] = kNoEdge;
        const int e = (int)(b & 0xffffffffu);
        M.in_msf[e] = 1;
        const int ep = M.epos ? M.epos[e] : e;
        int a = M.src[ep], c = M.col[ep];
        for (;;) {
            a = find_linking(M.parent, a);
            c = find_linking(M.parent, c);
            if (a == c) break;
            if (a < c) {
                const int t = a;
                a = c;
                c = t;
            }
            // a > c: hang root a under root c
            int expect = a;
            if (__hip_atomic_compare_exchange_strong(M.parent + a, &expect, c, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ++links;
                break;
            }
        }
    }
    msf_finish(M, KIND_AUX, 0, 0, links);
}

__global__ __launch_bounds__(256) void k_msf_compress(Msf M) {
    if (*(volatile int*)&M.ctl->done || *(volatile int*)&M.ctl->changed[M.r % 3] == 0) return;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    int* parent = M.parent;
    for (long long v = tid; v < M.n; v += tt) {
        int x = (int)v;
        int p = parent[x];
        while (p != x) {
            const int gp = parent[p];
            if (gp != p) parent[x] = gp;
            x = gp;
            p = parent[x];
        }
        parent[v] = x;
    }
}

__global__ __launch_bounds__(256) void k_msf_settle(Msf M) {
    if (*(volatile int*)&M.ctl->done || *(volatile int*)&M.ctl->changed[M.r % 3] == 0) return;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    const int* parent = M.parent;
    for (long long v = tid; v < M.n; v += tt) {
        int x = parent[v];
        while (parent[x] != x) x = parent[x];
        M.parent[v] = x;
    }
}

// Weight and edge count of the forest: one pair of 64-bit partial sums per
// block.
__global__ __launch_bounds__(256) void k_msf_sum(const unsigned char* in_msf, const int* w,
                                                 const int* epos, int m, long long* partial) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    long long sw = 0, cnt = 0;
    for (long long e = tid; e < m; e += tt)
        if (in_msf[e]) {
            sw += w[epos ? epos[e] : e];
            cnt++;
        }
    __shared__ long long s_w[4], s_c[4];
    for (int d = 32; d > 0; d >>= 1) {
        sw += __shfl_xor(sw, d, 64);
        cnt += __shfl_xor(cnt, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_w[threadIdx.x >> 6] = sw;
        s_c[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0, b = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            a += s_w[i];
            b += s_c[i];
        }
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

// Grid of a launch over `units` items, clamped to the blocks resident at once.
int msf_grid(const void* f, long long units) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, kBlock, 0) != hipSuccess || occ < 1)
        occ = 1;
    const long long cap = std::min<long long>((long long)occ * cus, kMaxStatBlocks);
    return (int)std::max(1LL, std::min<long long>((units + kBlock - 1) / kBlock, cap));
}

}  // namespace

extern "C" {

int gg_msf(gg_graph g, gg_ws ws, uint8_t* in_msf_dev, int64_t* total_weight, int64_t* n_edges,
           void* stream) {
    if (!g) return GG_EINVAL;
    if (g->err != GG_OK) return g->err;
    if (!ws) ws = g->ws0;
    if (ws->owner != g || !g->weighted || (g->m > 0 && !in_msf_dev)) return GG_EINVAL;
    WsClaim claim(ws);
    if (!claim.held()) return GG_EBUSY;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n = g->n;
    const int m = (int)g->m;
    // union-find and offers: kept in the workspace after the first call
    if (!ws->msf_parent) HIPCHK(g, dalloc(&ws->msf_parent, (size_t)n));
    if (!ws->msf_best) {
        void* p = nullptr;
        HIPCHK(g, hipMalloc(&p, sizeof(unsigned long long) * (size_t)n));
        ws->msf_best = static_cast<unsigned long long*>(p);
    }
    if (ws->used && ws->last_stream != s) HIPCHK(g, hipStreamWaitEvent(s, ws->finished, 0));
    hipError_t e = hipSuccess;
    const int tag = reserve_stamps(ws, s, kMsfMaxRounds + 2, &e);
    HIPCHK(g, e);
    Msf M{};
    M.src = g->src;
    M.col = g->col;
    M.w = g->w;
    M.eorig = g->renumbered ? g->eorig : nullptr;
    M.epos = g->renumbered ? g->epos : nullptr;
    M.n = n;
    M.m = m;
    M.parent = ws->msf_parent;
    M.best = ws->msf_best;
    M.in_msf = in_msf_dev;
    M.ctl = ws->dev.ctl;
    M.stat = ws->dev.stat;
    M.host_done = ws->h_done;
    M.tag = tag;
    const int g_init = msf_grid(reinterpret_cast<const void*>(k_msf_init), std::max(n, m));
    const int g_min = msf_grid(reinterpret_cast<const void*>(k_msf_min), (m + 3) / 4);
    const int g_vert = msf_grid(reinterpret_cast<const void*>(k_msf_link), n);
    hipLaunchKernelGGL(k_msf_init, dim3(g_init), dim3(kBlock), 0, s, M);
    HIPCHK(g, hipGetLastError());
    // batches of rounds, two outstanding, as in the traversal driver
    int r = 0, k = 0, status = GG_OK;
    auto enqueue = [&]() -> hipError_t {
        for (int i = 0; i < kMsfBatch && r < kMsfMaxRounds; ++i, ++r) {
            M.r = r;
            hipLaunchKernelGGL(k_msf_min, dim3(g_min), dim3(kBlock), 0, s, M);
            hipLaunchKernelGGL(k_msf_link, dim3(g_vert), dim3(kBlock), 0, s, M);
            hipLaunchKernelGGL(k_msf_compress, dim3(g_vert), dim3(kBlock), 0, s, M);
            hipLaunchKernelGGL(k_msf_settle, dim3(g_vert), dim3(kBlock), 0, s, M);
        }
        hipError_t x = hipGetLastError();
        if (x == hipSuccess) x = hipEventRecord(ws->ev[k & 1], s);
        ++k;
        return x;
    };
    auto reported = [&] { return __atomic_load_n(ws->h_done, __ATOMIC_ACQUIRE) == tag; };
    HIPCHK(g, enqueue());
    HIPCHK(g, enqueue());
    for (;;) {
        HIPCHK(g, hipEventSynchronize(ws->ev[k & 1]));
        if (reported()) break;
        if (r >= kMsfMaxRounds) {
            HIPCHK(g, hipEventSynchronize(ws->ev[(k + 1) & 1]));
            if (!reported()) status = GG_EITER;
            break;
        }
        HIPCHK(g, enqueue());
    }
    // forest weight and size
    long long* partial = reinterpret_cast<long long*>(ws->dev.pcount);
    const int g_sum = msf_grid(reinterpret_cast<const void*>(k_msf_sum), m);
    std::vector<long long> hp(2 * (size_t)g_sum);
    hipLaunchKernelGGL(k_msf_sum, dim3(g_sum), dim3(kBlock), 0, s, in_msf_dev, g->w, M.epos, m,
                       partial);
    HIPCHK(g, hipGetLastError());
    HIPCHK(g, hipMemcpyAsync(hp.data(), partial, sizeof(long long) * hp.size(),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(g, hipEventRecord(ws->finished, s));
    HIPCHK(g, hipEventSynchronize(ws->finished));
    long long tw = 0, cnt = 0;
    for (int i = 0; i < g_sum; ++i) {
        tw += hp[2 * (size_t)i];
        cnt += hp[2 * (size_t)i + 1];
    }
    if (total_weight) *total_weight = tw;
    if (n_edges) *n_edges = cnt;
    ws->rounds = r;
    ws->last_stream = s;
    ws->used = true;
    ws->profiled = false;
    ws->last = gg_stats{};
    ws->last.algo = GG_ALGO_MSF;
    ws->last.status = status;
    ws->last.grid_blocks = g_min;
    ws->last.block_threads = kBlock;
    return status;
}

}  // extern "C"
