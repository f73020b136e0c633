// gg_api.hip -- host runtime and C ABI of libgg (declared in include/gg.h).
//
// A traversal is an init kernel followed by rounds (one kernel each, plus a
// heavy-chunk kernel or a CC shortcut kernel where the variant needs one).
// The host enqueues rounds in batches that double in size up to kMaxBatch;
// after each batch it copies the device `done` flag into pinned memory and
// records an event.  While batch k runs, the host waits for batch k-1's event
// and stops enqueueing once that batch reported `done`.  Rounds enqueued past
// the end return at their first instruction, so the overshoot costs at most
// one batch of empty launches.

#include <gg.h>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "gg_internal.h"
#include "gg_runtime.h"

using namespace gg;


namespace {

// Heavy-row chunks of a CSR held on the host, in row order.
std::vector<int2> build_chunks(const std::vector<int>& row, int n, int heavy, int chunk) {
    std::vector<int2> out;
    for (int v = 0; v < n; ++v) {
        const int d = row[v + 1] - row[v];
        if (d > heavy)
            for (int e = row[v]; e < row[v + 1]; e += chunk) out.push_back(make_int2(v, e));
    }
    return out;
}

int grid_for(long long items_per_block_unit, long long units) {
    (void)items_per_block_unit;
    const long long cap = device().max_blocks;
    long long g = units;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void free_ws_arrays(gg_ws_s* ws) {
    if (!ws) return;
    if (ws->vflag_mem) (void)hipFree(ws->vflag_mem);
    if (ws->dev.hbits[0]) (void)hipFree(ws->dev.hbits[0]);
    if (ws->dev.ctl) (void)hipFree(ws->dev.ctl);
    if (ws->dev.stat) (void)hipFree(ws->dev.stat);
    if (ws->dev.pcount) (void)hipFree(ws->dev.pcount);
    if (ws->h_done) (void)hipHostFree(ws->h_done);
    if (ws->msf_parent) (void)hipFree(ws->msf_parent);
    if (ws->msf_best) (void)hipFree(ws->msf_best);
    ws->msf_parent = nullptr;
    ws->msf_best = nullptr;
    dfree(ws->rval);
    dfree(ws->rmin);
    for (auto& e : ws->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ws->pev)
        if (e) (void)hipEventDestroy(e);
    ws->pev.clear();
    if (ws->finished) (void)hipEventDestroy(ws->finished);
    ws->vflag_mem = nullptr;
    ws->dev.hbits[0] = ws->dev.hbits[1] = nullptr;
    ws->dev.ctl = nullptr;
    ws->dev.stat = nullptr;
    ws->h_done = nullptr;
}

int make_ws(gg_graph g, gg_ws_s** out) {
    gg_ws_s* ws = new (std::nothrow) gg_ws_s();
    if (!ws) return GG_ENOMEM;
    ws->owner = g;
    const long long ntiles = (g->n + 63) / 64;
    // vertex flags padded to whole 64-tile groups so no index needs a bound
    const long long vbytes = ((ntiles + 63) / 64) * 64 * 64;
    const long long tbytes = ((ntiles + 63) / 64) * 64;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(&ws->vflag_mem, (size_t)(2 * (vbytes + tbytes)));
    const long long hwords = ((long long)g->n + 31) / 32;
    if (e == hipSuccess) e = dalloc(&ws->dev.hbits[0], (size_t)(2 * hwords));
    if (e == hipSuccess) e = hipMemset(ws->dev.hbits[0], 0, sizeof(unsigned) * (size_t)(2 * hwords));
    if (e == hipSuccess) e = dalloc(&ws->dev.ctl, 1);
    if (e == hipSuccess) e = dalloc(&ws->dev.stat, (size_t)kKinds * kMaxStatBlocks);
    if (e == hipSuccess) e = dalloc(&ws->dev.pcount, (size_t)3 * 2 * kMaxStatBlocks);
    if (e == hipSuccess && g->renumbered) e = dalloc(&ws->rval, (size_t)g->n);
    if (e == hipSuccess && g->renumbered) e = dalloc(&ws->rmin, (size_t)g->n);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ws->h_done), 4 * sizeof(int));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->ev[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->finished, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemset(ws->vflag_mem, 0, (size_t)(2 * (vbytes + tbytes)));
    if (e == hipSuccess) e = hipMemset(ws->dev.ctl, 0, sizeof(Ctl));
    // the fills above are queued on the null stream and may still be in
    // flight when hipMemset returns; traversals use the workspace on other
    // (non-blocking) streams, which do not wait for the null stream: wait
    // here, so that a fill can never land in the middle of a traversal
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        free_ws_arrays(ws);
        delete ws;
        return fail_hip(g, e);
    }
    ws->dev.hbits[1] = ws->dev.hbits[0] + hwords;
    ws->dev.vflag[0] = ws->vflag_mem;
    ws->dev.vflag[1] = ws->vflag_mem + vbytes;
    ws->dev.tflag[0] = ws->vflag_mem + 2 * vbytes;
    ws->dev.tflag[1] = ws->vflag_mem + 2 * vbytes + tbytes;
    ws->h_done[0] = -1;
    *prog_word(ws) = 0;
    *out = ws;
    return GG_OK;
}

// Upload checks of host edge arrays, split over host threads: every column
// in [0, n), every weight >= 0; the largest weight and the weight sum.
struct HostCheck {
    bool ok = true;
    int max_w = 0;
    long long wsum = 0;
};

HostCheck check_host(const int* col, const int* w, long long m, int n) {
    const int nt = (int)std::max(1LL, std::min<long long>(
                            std::min<long long>(16, std::thread::hardware_concurrency()),
                            m / (1 << 20) + 1));
    std::vector<HostCheck> part((size_t)nt);
    auto work = [&](int t) {
        HostCheck& r = part[(size_t)t];
        const long long e0 = m * t / nt, e1 = m * (t + 1) / nt;
        for (long long e = e0; e < e1; ++e)
            if ((unsigned)col[e] >= (unsigned)n) r.ok = false;
        if (w)
            for (long long e = e0; e < e1; ++e) {
                const int x = w[e];
                if (x < 0) r.ok = false;
                r.max_w = std::max(r.max_w, x);
                r.wsum += x;
            }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) {
        try {
            th.emplace_back(work, t);
        } catch (...) {
            work(t);  // no thread: check the part here
        }
    }
    work(0);
    for (auto& x : th) x.join();
    HostCheck r;
    for (const HostCheck& x : part) {
        r.ok = r.ok && x.ok;
        r.max_w = std::max(r.max_w, x.max_w);
        r.wsum += x.wsum;
    }
    return r;
}

// Graphs with fewer edges keep the single edge list for the edge sweep.
constexpr long long kPartMinEdges = 1LL << 20;

// Renumber an uploaded CSR (device row/col/w of the handle; hrow, the host
// copy of the offsets): new ids by descending total degree, ties in the
// caller's order (a stable counting sort on the host), each row's edges
// then ordered by head (sort_rows_by_head).  Leaves the renumbered arrays
// in the handle, hrow and hin
// (in-degrees) in the new order, the id maps, and -- for a weighted graph,
// the only kind a forest is built on -- the edge maps.  tmp: n + 8 ints.
int renumber_graph(gg_graph g, std::vector<int>& hrow, std::vector<int>& hin, int* tmp,
                   hipStream_t s) {
    const int n = g->n;
    const long long m = g->m;
    auto grid = [&](long long units) {
        return (int)std::max(1LL, std::min<long long>(units, device().max_blocks));
    };
    hin.assign((size_t)n, 0);
    hipError_t e = hipMemsetAsync(tmp, 0, sizeof(int) * n, s);
    if (e == hipSuccess)
        e = launch_count_in(g->col, (int)m, tmp, grid((m + kBlock - 1) / kBlock), kBlock, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hin.data(), tmp, sizeof(int) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return GG_EHIP;
    // keys (out + in degree, < 2^32) and the order: counting sort when the
    // largest key is small against n, else a stable comparison sort
    std::vector<long long> key((size_t)n);
    long long kmax = 0;
    for (int v = 0; v < n; ++v) {
        key[v] = (long long)(hrow[v + 1] - hrow[v]) + hin[v];
        kmax = std::max(kmax, key[v]);
    }
    std::vector<int> oldid((size_t)n), newid((size_t)n);
    if (kmax <= 4LL * n + 1024) {
        std::vector<int> start((size_t)kmax + 2, 0);
        for (int v = 0; v < n; ++v) start[(size_t)(kmax - key[v]) + 1]++;
        for (long long k = 1; k <= kmax + 1; ++k) start[(size_t)k] += start[(size_t)k - 1];
        for (int v = 0; v < n; ++v) oldid[(size_t)start[(size_t)(kmax - key[v])]++] = v;
    } else {
        for (int v = 0; v < n; ++v) oldid[v] = v;
        std::stable_sort(oldid.begin(), oldid.end(),
                         [&](int a, int b) { return key[a] > key[b]; });
    }
    for (int k = 0; k < n; ++k) newid[(size_t)oldid[k]] = k;
    // vertices without any edge come last
    int active = n;
    while (active > 0 && key[(size_t)oldid[(size_t)active - 1]] == 0) --active;
    std::vector<int> nrow((size_t)n + 1), nin((size_t)n);
    nrow[0] = 0;
    for (int k = 0; k < n; ++k) {
        const int u = oldid[k];
        nrow[(size_t)k + 1] = nrow[k] + (hrow[(size_t)u + 1] - hrow[u]);
        nin[k] = hin[(size_t)u];
    }
    int *drow = nullptr, *dcol = nullptr, *dw = nullptr;
    auto fail = [&](hipError_t x) {
        (void)hipStreamSynchronize(s);
        dfree(drow);
        dfree(dcol);
        dfree(dw);
        return x == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP;
    };
    e = dalloc(&g->newid, (size_t)n);
    if (e == hipSuccess) e = dalloc(&g->oldid, (size_t)n);
    if (e == hipSuccess) e = dalloc(&drow, (size_t)n + 1);
    if (e == hipSuccess) e = dalloc(&dcol, (size_t)m);
    if (e == hipSuccess && g->w) e = dalloc(&dw, (size_t)m);
    if (e == hipSuccess && g->w) e = dalloc(&g->eorig, (size_t)m);
    if (e == hipSuccess && g->w) e = dalloc(&g->epos, (size_t)m);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->newid, newid.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->oldid, oldid.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(drow, nrow.data(), sizeof(int) * ((size_t)n + 1), hipMemcpyHostToDevice, s);
    // the caller's edge sources, then every edge to its new place
    if (e == hipSuccess)
        e = launch_fill_src(g->row, n, (int)m, g->src, grid((m + 4095) / 4096), kBlock, s);
    if (e == hipSuccess)
        e = launch_renumber(g->row, g->col, g->w, g->src, (int)m, g->newid, drow, dcol, dw,
                            g->eorig, g->epos, grid((m + kBlock - 1) / kBlock), kBlock, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(e);
    dfree(g->row);
    dfree(g->col);
    dfree(g->w);
    g->row = drow;
    g->col = dcol;
    g->w = dw;
    // each row's edges by head: the gathers of a long row share lines
    const int rc = sort_rows_by_head(g, s);
    if (rc != GG_OK) return rc;
    hrow.swap(nrow);
    hin.swap(nin);
    g->h_newid.swap(newid);
    g->renumbered = true;
    g->n_active = active;
    return GG_OK;
}

// The edge list again, cut into kXcd parts by head vertex with equal edge
// counts (part boundaries at the in-degree quantiles), CSR order kept inside
// a part, each part padded to a multiple of 4 edges with the self-loop 0->0
// of weight 0 (it never changes a value).  The split runs on the device
// (per-block counts per part, bases from their prefix sums on the host, then
// a stable placement); hin holds the in-degrees.
int build_parts(gg_graph g, const std::vector<int>& hin, hipStream_t s) {
    const int n = g->n;
    const long long m = g->m;
    std::vector<unsigned char> part((size_t)n);
    long long cum = 0;
    int p = 0;
    for (int v = 0; v < n; ++v) {
        while (p < kXcd - 1 && cum >= (long long)(p + 1) * m / kXcd) ++p;
        part[v] = (unsigned char)p;
        cum += hin[v];
    }
    const int nb = split_blocks(m);
    unsigned char* dpart = nullptr;
    int* dcounts = nullptr;
    long long* dbase = nullptr;
    std::vector<int> counts((size_t)nb * kXcd);
    auto done = [&](int rc) {
        dfree(dpart);
        dfree(dcounts);
        dfree(dbase);
        return rc;
    };
    hipError_t e = dalloc(&dpart, (size_t)n);
    if (e == hipSuccess) e = dalloc(&dcounts, counts.size());
    if (e == hipSuccess) e = hipMemcpyAsync(dpart, part.data(), (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_split_count(g->col, (int)m, dpart, dcounts, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts.data(), dcounts, sizeof(int) * counts.size(),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP);
    long long cnt[kXcd] = {};
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < kXcd; ++k) cnt[k] += counts[(size_t)b * kXcd + k];
    long long off[kXcd + 1];
    off[0] = 0;
    for (int k = 0; k < kXcd; ++k) off[k + 1] = off[k] + ((cnt[k] + 3) & ~3LL);
    const long long mp = off[kXcd];
    if (mp >= (1LL << 31)) return done(GG_OK);  // keep the single list
    std::vector<long long> base((size_t)nb * kXcd);
    long long run[kXcd];
    for (int k = 0; k < kXcd; ++k) run[k] = off[k];
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < kXcd; ++k) {
            base[(size_t)b * kXcd + k] = run[k];
            run[k] += counts[(size_t)b * kXcd + k];
        }
    e = dalloc(&dbase, base.size());
    if (e == hipSuccess) e = dalloc(&g->psrc, (size_t)mp);
    if (e == hipSuccess) e = dalloc(&g->pcol, (size_t)mp);
    if (e == hipSuccess && g->w) e = dalloc(&g->pw, (size_t)mp);
    // the padding edges are the zero self-loop 0->0
    if (e == hipSuccess) e = hipMemsetAsync(g->psrc, 0, sizeof(int) * mp, s);
    if (e == hipSuccess) e = hipMemsetAsync(g->pcol, 0, sizeof(int) * mp, s);
    if (e == hipSuccess && g->w) e = hipMemsetAsync(g->pw, 0, sizeof(int) * mp, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dbase, base.data(), sizeof(long long) * base.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_split_place(g->src, g->col, g->w, (int)m, dpart, dbase, g->psrc, g->pcol,
                               g->pw, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        dfree(g->psrc);
        dfree(g->pcol);
        dfree(g->pw);
        return done(e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP);
    }
    for (int k = 0; k <= kXcd; ++k) g->poff[k] = (int)off[k];
    return done(GG_OK);
}

void free_graph_arrays(gg_graph g) {
    dfree(g->trow);
    dfree(g->tcol);
    dfree(g->tw);
    dfree(g->tchunks);
    dfree(g->psrc);
    dfree(g->pcol);
    dfree(g->pw);
    if (g->srow && g->srow != g->row) (void)hipFree(g->srow);
    if (g->scol && g->scol != g->col) (void)hipFree(g->scol);
    if (g->ssrc && g->ssrc != g->src) (void)hipFree(g->ssrc);
    dfree(g->row);
    dfree(g->col);
    dfree(g->w);
    dfree(g->src);
    dfree(g->hchunks);
    dfree(g->shchunks);
    dfree(g->newid);
    dfree(g->oldid);
    dfree(g->eorig);
    dfree(g->epos);
    g->srow = g->scol = g->ssrc = nullptr;
}

DevGraph dev_graph(gg_graph g) {
    DevGraph d{};
    d.n = g->n;
    d.m = (int)g->m;
    d.row = g->row;
    d.col = g->col;
    d.w = g->w;
    d.src = g->src;
    d.ms = (int)g->ms;
    d.srow = g->srow;
    d.scol = g->scol;
    d.ssrc = g->ssrc;
    d.heavy = g->heavy;
    d.chunk = g->chunk;
    d.hchunks = g->hchunks;
    d.n_hchunks = g->n_hchunks;
    d.shchunks = g->shchunks;
    d.n_shchunks = g->n_shchunks;
    d.symmetric = g->symmetric;
    d.psrc = g->psrc;
    d.pcol = g->pcol;
    d.pw = g->pw;
    for (int k = 0; k <= kXcd; ++k) d.poff[k] = g->poff[k];
    d.trow = g->trow;
    d.tcol = g->tcol;
    d.tw = g->tw;
    d.tchunks = g->tchunks;
    d.n_tchunks = g->n_tchunks;
    return d;
}

// The per-round dense/sparse schedule: BFS vertex-based (pull over
// in-neighbours), CC edge-based (dense rounds sweep the stored edges) or
// vertex-based (dense rounds pull over the both-directions rows) -- these
// read the both-directions CSR -- and SSSP vertex-based (dense rounds pull
// over the weighted in-edge CSR).
bool diropt_ok(gg_graph g, int algo, int mode) {
    if (algo == GG_ALGO_SSSP) return mode == GG_VERTEX && g->trow != nullptr;
    if (!g->has_sym) return false;
    return (algo == GG_ALGO_BFS && mode == GG_VERTEX) ||
           (algo == GG_ALGO_CC && (mode == GG_EDGE || mode == GG_VERTEX));
}

// AUTO fields resolve through the tuning table (else built-in rules) for
// the graph's class; explicit fields are kept.
void resolve(gg_graph g, int algo, const gg_opts* in, gg_opts* out) {
    // no options: the tuned choice of every field
    gg_opts o{};
    o.mode = GG_MODE_AUTO;
    o.sched = GG_SCHED_AUTO;
    o.mapping = GG_MAP_AUTO;
    if (in) o = *in;
    const bool auto_mode = o.mode != GG_VERTEX && o.mode != GG_EDGE;
    const bool auto_sched = o.sched != GG_SYNC && o.sched != GG_ASYNC && o.sched != GG_NEARFAR &&
                            o.sched != GG_DIROPT && o.sched != GG_UNIONFIND;
    const bool auto_map = o.mapping < GG_MAP_THREAD || o.mapping > GG_MAP_BALANCED;
    int32_t sc = 0, kc = 0, dc = -1;
    gg_class_of(g->m, g->n, g->max_deg, g->levels, &sc, &kc, &dc);
    gg_tune_entry t{};
    t.mode = GG_VERTEX;
    t.sched = GG_ASYNC;
    t.mapping = GG_MAP_BALANCED;
    gg_tune_lookup(algo, sc, kc, dc, &t);
    const int32_t tm = t.mode, ts = t.sched, tp = t.mapping, te = t.delta_eighths;
    if (auto_mode) o.mode = tm;
    // the tuned schedule comes with its local expansion and deferral
    if (auto_sched) {
        o.sched = ts;
        o.hops = t.hops;
        o.far_degree = t.far_degree;
    }
    // an explicit per-round schedule fixes the mode it runs in
    if (!auto_sched && o.sched == GG_DIROPT && auto_mode)
        o.mode = algo == GG_ALGO_CC ? GG_EDGE : GG_VERTEX;
    if (auto_map) o.mapping = tp;
    // bucket width of the near-far schedule: explicit, else the table's
    // eighths of the mean weight, else 4 mean weights
    // (computed in double and capped at 2^30 before the conversion: with
    // weights near 2^31 the product passes the int range, and the bound
    // saturates at INF long before a width of 2^30 matters)
    if (o.sched == GG_NEARFAR && o.delta <= 0) {
        const double d = (te > 0 ? te : 32) * g->avg_w / 8.0;
        o.delta = d >= (double)(1 << 30) ? (1 << 30) : std::max(1, (int)d);
    }
    // a choice taken from the table must be one this graph can run
    if (auto_sched && o.sched == GG_DIROPT && !diropt_ok(g, algo, o.mode)) {
        o.sched = algo == GG_ALGO_CC ? GG_SYNC : GG_ASYNC;
        if (algo == GG_ALGO_CC && auto_mode) o.mode = GG_EDGE;
    }
    if (auto_sched && o.sched == GG_NEARFAR && (algo != GG_ALGO_SSSP || o.mode != GG_VERTEX))
        o.sched = GG_ASYNC;
    if (auto_sched && o.sched == GG_UNIONFIND && (algo != GG_ALGO_CC || !g->has_sym)) {
        o.sched = algo == GG_ALGO_CC ? GG_SYNC : GG_ASYNC;
        if (algo == GG_ALGO_CC && auto_mode) o.mode = GG_EDGE;
    }
    // an explicit union-find schedule runs vertex-based
    if (!auto_sched && o.sched == GG_UNIONFIND && auto_mode) o.mode = GG_VERTEX;
    // without the both-directions CSR only the edge sweep can run CC
    if (algo == GG_ALGO_CC && !g->has_sym) {
        if (auto_mode) o.mode = GG_EDGE;
        if (auto_sched) o.sched = GG_SYNC;
    }
    if (o.block_threads <= 0) o.block_threads = kBlock;
    if (o.time_limit_ms <= 0) o.time_limit_ms = kDefaultTimeLimitMs;
    *out = o;
}

}  // namespace

namespace gg {

int plan_make(gg_graph g, gg_ws ws, int algo, int source, const int* sources_dev, int nsrc,
              const gg_opts* opts, int* out, hipStream_t s, Plan* P) {
    if (!g) return GG_EINVAL;
    if (g->err != GG_OK) return g->err;
    if (!out || nsrc < 0 || (nsrc > 0 && !sources_dev)) return GG_EINVAL;
    if (algo != GG_ALGO_CC && nsrc == 0 && (source < 0 || source >= g->n)) return GG_EINVAL;
    if (algo == GG_ALGO_SSSP && !g->weighted) return GG_EINVAL;
    if (!ws) ws = g->ws0;
    if (ws->owner != g) return GG_EINVAL;
    Plan& p = *P;
    p = Plan{};
    p.g = g;
    p.ws = ws;
    p.algo = algo;
    p.s = s;
    resolve(g, algo, opts, &p.o);
    const gg_opts& o = p.o;
    // CC reads the both-directions CSR except in the synchronous edge sweep
    if (algo == GG_ALGO_CC && !g->has_sym && (o.mode != GG_EDGE || o.sched != GG_SYNC))
        return GG_ENOTSUP;
    if (o.block_threads != kBlock) return GG_ENOTSUP;
    const bool nearfar = o.sched == GG_NEARFAR;
    if (nearfar && (algo != GG_ALGO_SSSP || o.mode != GG_VERTEX || o.mapping != GG_MAP_BALANCED))
        return GG_ENOTSUP;
    if (o.delta < 0 || o.hops < 0 || o.hops > 64 || o.far_degree < 0) return GG_EINVAL;
    const bool diropt = o.sched == GG_DIROPT;
    if (diropt && !diropt_ok(g, algo, o.mode)) return GG_ENOTSUP;
    const bool uf = o.sched == GG_UNIONFIND;
    if (uf && (algo != GG_ALGO_CC || o.mode != GG_VERTEX || !g->has_sym)) return GG_ENOTSUP;
    const Dev& dv = device();
    const int cap_blocks = o.max_blocks > 0 ? std::min(o.max_blocks, dv.max_blocks) : dv.max_blocks;
    auto grid = [&](long long units) {
        return (int)std::max(1LL, std::min<long long>(units, cap_blocks));
    };
    p.async = o.sched == GG_ASYNC || nearfar || diropt;
    p.diropt = diropt;
    p.uf = uf;
    p.edge = o.mode == GG_EDGE;
    p.cc = algo == GG_ALGO_CC;
    Round& R = p.R;
    R.g = dev_graph(g);
    R.ws = ws->dev;
    R.val = out;
    R.source = p.cc ? 0 : source;
    if (g->renumbered) {
        // multi-source traversals (batches) run on graphs in the caller's order
        if (nsrc > 0) return GG_ENOTSUP;
        p.renum = true;
        p.out = out;
        p.src_caller = p.cc ? -1 : source;
        R.val = ws->rval;
        if (!p.cc) R.source = g->h_newid[(size_t)source];
        if (p.cc) R.rmin = ws->rmin;
    }
    R.sources = sources_dev;
    R.nsrc = p.cc ? 0 : nsrc;
    R.mapping = o.mapping;
    R.jump = p.cc && !(o.flags & GG_OPT_CC_NO_JUMP);
    R.host_done = ws->h_done;
    // default bucket width: a few mean weights (one bucket then spans paths
    // of several light edges)
    R.delta = nearfar ? std::max(1, o.delta) : 0;
    R.fedges = diropt && (p.cc || algo == GG_ALGO_SSSP);
    R.pullmode = diropt && (algo == GG_ALGO_SSSP || (p.cc && o.mode == GG_VERTEX));
    R.hops = p.async && !p.edge && !diropt && o.mapping == GG_MAP_BALANCED ? o.hops : 0;
    R.far_degree = nearfar ? o.far_degree : 0;
    R.direct_lists = (o.flags & GG_OPT_LISTS_DIRECT)    ? 1
                     : (o.flags & GG_OPT_LISTS_CHECKED) ? 0
                                                         : (g->levels >= 256 ? 1 : 0);

    const int wpb = kBlock / 64;
    const long long n = g->n;
    const long long ntiles = (n + 63) / 64;
    const long long ngroups = (ntiles + 63) / 64;
    const int nh = p.cc ? g->n_shchunks : g->n_hchunks;
    p.g_init = grid((n + kBlock - 1) / kBlock);
    p.g_seed = grid((nsrc + kBlock - 1) / kBlock);
    if (!p.async && !p.edge) {
        if (o.mapping == GG_MAP_BALANCED) p.g_round = grid((nh + ntiles + wpb - 1) / wpb);
        else if (o.mapping == GG_MAP_THREAD) p.g_round = grid((n + kBlock - 1) / kBlock);
        else p.g_round = grid((n + wpb - 1) / wpb);
    } else if (!p.async && p.edge) {
        p.g_round = grid((g->m / 4 + kBlock - 1) / kBlock);
    } else if (diropt && p.cc) {
        p.g_round = grid(std::max(ngroups * kParts / wpb + 1, (g->m / 4 + kBlock - 1) / kBlock));
    } else if (diropt && algo == GG_ALGO_SSSP) {
        p.g_round = grid(std::max(ngroups * kParts, ntiles + g->n_tchunks) / wpb + 1);
    } else if (diropt) {
        p.g_round = grid(std::max(ngroups * kParts, ntiles) / wpb + 1);
    } else if (uf) {
        p.g_round = grid((n + kBlock - 1) / kBlock);
    } else {
        p.g_round = grid((ngroups * kParts + wpb - 1) / wpb);
    }
    p.need_heavy = p.async && (p.edge || diropt || o.mapping == GG_MAP_BALANCED) && nh > 0;
    // the heavy kernel of an SSSP pull round clears the frontier it read
    if (diropt && algo == GG_ALGO_SSSP) p.need_heavy = true;
    p.g_heavy = grid((nh + 64LL * wpb - 1) / (64LL * wpb));
    if (diropt && algo == GG_ALGO_SSSP)  // enough blocks to clear the flags quickly
        p.g_heavy = std::max(p.g_heavy, grid((ngroups * 256 + kBlock - 1) / kBlock));
    p.need_jump = p.cc && p.edge && (!p.async || diropt) && R.jump && !uf;
    // ... and the shortcut kernel of a CC pull round
    if (diropt && p.cc && R.pullmode) p.need_jump = true;
    p.g_jump = grid((n + kBlock - 1) / kBlock);
    return GG_OK;
}

// Reference point of the profiled time line: an event recorded on the
// stream of the first profiled call of the process.
hipEvent_t g_time_ref = nullptr;
std::once_flag g_time_ref_once;

// Every launch goes through here so that profiling can bracket it.
template <class F>
hipError_t plan_launch(Plan& p, int kind, F&& fn) {
    gg_ws ws = p.ws;
    if (!p.prof) return fn();
    hipError_t e = hipSuccess;
    std::call_once(g_time_ref_once, [&] {
        if (hipEventCreate(&g_time_ref) == hipSuccess &&
            hipEventRecord(g_time_ref, p.s) != hipSuccess) {
            (void)hipEventDestroy(g_time_ref);
            g_time_ref = nullptr;
        }
    });
    const int i = ws->nlaunch;
    while ((int)ws->pev.size() < 2 * (i + 1)) {
        hipEvent_t ev;
        e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
        ws->pev.push_back(ev);
    }
    if ((int)ws->pkind.size() < i + 1) ws->pkind.resize(i + 1);
    e = hipEventRecord(ws->pev[2 * i], p.s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e == hipSuccess) {
        e = hipEventRecord(ws->pev[2 * i + 1], p.s);
        ws->pkind[i] = kind;
        ws->nlaunch = i + 1;
    }
    return e;
}

hipError_t plan_init(Plan& p) {
    hipError_t e = plan_launch(p, KIND_AUX, [&] {
        return launch_init(p.R, p.algo, p.async, p.g_init, kBlock, p.s);
    });
    if (e == hipSuccess && p.R.nsrc > 0)
        e = plan_launch(p, KIND_AUX, [&] { return launch_seed(p.R, p.async, p.g_seed, kBlock, p.s); });
    return e;
}

// Round r of the plan's traversal.
hipError_t plan_round(Plan& p, int r) {
    Round& R = p.R;
    R.r = r;
    hipError_t e = plan_launch(p, KIND_ROUND, [&] {
        if (p.uf) return launch_uf(R, p.g_round, kBlock, p.s);
        if (p.diropt && p.cc) return launch_cc_diropt(R, p.g_round, kBlock, p.s);
        if (p.diropt && p.algo == GG_ALGO_SSSP) return launch_sssp_diropt(R, p.g_round, kBlock, p.s);
        if (p.diropt) return launch_bfs_diropt(R, p.g_round, kBlock, p.s);
        if (!p.async && !p.edge) return launch_vsync(R, p.algo, p.g_round, kBlock, p.s);
        if (!p.async) return launch_esync(R, p.algo, p.g_round, kBlock, p.s);
        if (!p.edge) return launch_vasync(R, p.algo, p.g_round, kBlock, p.s);
        return launch_easync(R, p.algo, p.g_round, kBlock, p.s);
    });
    if (e == hipSuccess && p.need_heavy)
        e = plan_launch(p, KIND_HEAVY, [&] { return launch_heavy(R, p.algo, p.g_heavy, kBlock, p.s); });
    if (e == hipSuccess && p.need_jump)
        e = plan_launch(p, KIND_AUX, [&] { return launch_jump(R, p.g_jump, kBlock, p.s); });
    // union-find: a compression after each linking phase
    if (e == hipSuccess && p.uf && r != 2 && r <= 3)
        e = plan_launch(p, KIND_AUX, [&] { return launch_uf_compress(R, p.g_round, kBlock, p.s); });
    return e;
}

hipError_t plan_finish(Plan& p) {
    if (!p.renum) return hipSuccess;
    gg_graph g = p.g;
    const int n = g->n;
    const int gv = (int)std::max(1LL, std::min<long long>((n + kBlock - 1) / kBlock,
                                                          device().max_blocks));
    // a vertex without edges (new id >= n_active) is its own component and
    // reached only as the source: its value needs no gather
    const int na = g->n_active;
    if (p.cc) {
        // about 64 new ids per lane for the running minimum
        const int gm = (int)std::max(1LL, std::min<long long>((na + 64LL * kBlock - 1) /
                                                              (64LL * kBlock), device().cus));
        hipError_t e = hipSuccess;
        if (na > 0)
            e = plan_launch(p, KIND_AUX, [&] {
                return launch_cc_min_ids(p.R.val, g->oldid, p.R.rmin, na, gm, kBlock, p.s);
            });
        if (e != hipSuccess) return e;
        return plan_launch(p, KIND_AUX, [&] {
            return launch_cc_min_out(p.out, p.R.val, g->newid, p.R.rmin, n, na, gv, kBlock, p.s);
        });
    }
    return plan_launch(p, KIND_AUX, [&] {
        return launch_unrenumber(p.out, p.R.val, g->newid, n, na, p.src_caller, gv, kBlock, p.s);
    });
}

// Reserve `span` round stamps on the workspace; returns the first.  The
// first stamp of a traversal is its tag: the round kernel that finds the end
// stores it into the workspace's pinned word, so a late kernel of an earlier
// traversal (an older, smaller tag) cannot end this one.  Stamps restart
// long before the 32-bit range ends (the previous tag is then large).
int reserve_stamps(gg_ws ws, hipStream_t s, long long span, hipError_t* err) {
    (void)s;
    *err = hipSuccess;
    if ((long long)ws->epoch + span > (1LL << 30)) ws->epoch = 0;
    const int base = ws->epoch;
    ws->epoch = (int)std::min<long long>((long long)base + span, 1LL << 30);
    return base;
}

// Eager driver as a resumable state machine.  Batches of rounds double in
// size up to kMaxBatch; at most two batches are outstanding.  When the older
// one has completed, the pinned word tells whether some round kernel found
// the end (it stores the traversal's tag); if not, the next batch goes out.
// Rounds enqueued past the end return at their first instruction.
// Bound on the rounds of a traversal.  Every round of a sweep or worklist
// schedule that changes something fixes at least one more vertex, so n + 2
// rounds suffice; a near-far round may only raise the bound, which happens
// at most (largest possible distance) / delta times.
long long max_rounds(const Plan& p) {
    long long r = (long long)p.g->n + 2;
    if (p.R.delta > 0)
        r += std::min<long long>(((long long)p.g->n * p.g->max_w) / p.R.delta + 1, 1LL << 29);
    return std::min(r, 1LL << 30);
}

int drive_start(Drive& d, long long r0, int stamp_base, int tag) {
    d.r = r0;
    d.batch = 2;
    d.k = 0;
    d.stamp_base = stamp_base;
    d.tag = tag;
    d.max_rounds = max_rounds(d.p);
    d.t0 = std::chrono::steady_clock::now();
    d.status = GG_OK;
    d.finished = false;
    d.stopping = false;
    d.finishing = false;
    d.fin_seq = 0;
    // two batches in flight from the start
    for (int i = 0; i < 2; ++i) {
        int rc = drive_enqueue(d);
        if (rc != GG_OK) return rc;
    }
    return GG_OK;
}

int drive_enqueue(Drive& d) {
    Plan& p = d.p;
    const long long stop = std::min(d.r + d.batch, d.max_rounds);
    for (; d.r < stop; ++d.r) HIPCHK(p.g, plan_round(p, (int)d.r));
    if (d.poll) {
        const unsigned long long v = ++p.ws->prog_seq;
        HIPCHK(p.g, launch_mark(prog_word(p.ws), v, p.s));
        d.seq[d.k & 1] = v;
    } else {
        HIPCHK(p.g, hipEventRecord(p.ws->ev[d.k & 1], p.s));
    }
    ++d.k;
    d.batch = std::min(d.batch * 2, kMaxBatch);
    return GG_OK;
}

// The rounds are over (the end was reported, or rounds or time ran out).
// Without finishing kernels the traversal is finished now; otherwise they
// are enqueued once, followed by a marker (polled) or an event, and the
// traversal is finished when that has run: its output is then complete.
int drive_end(Drive& d, bool block) {
    Plan& p = d.p;
    gg_ws ws = p.ws;
    if (!p.renum) {
        d.finished = true;
        return 1;
    }
    if (!d.finishing) {
        HIPCHK(p.g, plan_finish(p));
        d.finishing = true;
        if (d.poll) {
            d.fin_seq = ++ws->prog_seq;
            HIPCHK(p.g, launch_mark(prog_word(ws), d.fin_seq, p.s));
        } else {
            // the older batch's event has completed: its slot is free
            HIPCHK(p.g, hipEventRecord(ws->ev[d.k & 1], p.s));
        }
    }
    if (d.poll) {
        if (__atomic_load_n(prog_word(ws), __ATOMIC_ACQUIRE) < d.fin_seq) return 0;
    } else if (block) {
        HIPCHK(p.g, hipEventSynchronize(ws->ev[d.k & 1]));
    } else {
        const hipError_t q = hipEventQuery(ws->ev[d.k & 1]);
        if (q == hipErrorNotReady) return 0;
        HIPCHK(p.g, q);
    }
    d.finished = true;
    return 1;
}

int drive_step(Drive& d, bool block) {
    if (d.finished) return 1;
    if (d.finishing) return drive_end(d, block);
    Plan& p = d.p;
    gg_ws ws = p.ws;
    auto reported = [&] { return __atomic_load_n(ws->h_done, __ATOMIC_ACQUIRE) == d.tag; };
    auto completed = [&](int slot) { return __atomic_load_n(prog_word(ws), __ATOMIC_ACQUIRE) >= d.seq[slot]; };
    // batch k-2 is the older of the two outstanding (k-1 the newer one)
    if (d.poll) {
        if (reported()) {
            // the values are final once the end is found; rounds still queued
            // return at their first instruction
            return drive_end(d, block);
        }
        if (d.stopping) {
            // out of rounds or time: the newer batch must complete before the
            // status is final (checked on later steps, never waited for here)
            if (!completed((d.k + 1) & 1)) return 0;
            if (!reported()) d.status = d.stop_status;
            return drive_end(d, block);
        }
        if (!completed(d.k & 1)) return 0;
    } else if (block) {
        HIPCHK(p.g, hipEventSynchronize(ws->ev[d.k & 1]));
    } else {
        const hipError_t q = hipEventQuery(ws->ev[d.k & 1]);
        if (q == hipErrorNotReady) return 0;
        HIPCHK(p.g, q);
    }
    if (reported()) return drive_end(d, block);
    const long long ms = std::chrono::duration_cast<std::chrono::milliseconds>(
                             std::chrono::steady_clock::now() - d.t0).count();
    if (d.r >= d.max_rounds || ms > p.o.time_limit_ms) {
        const int st = d.r >= d.max_rounds ? GG_EITER : GG_ETIMEOUT;
        if (d.poll) {
            d.stopping = true;
            d.stop_status = st;
            if (!completed((d.k + 1) & 1)) return 0;
        } else {
            HIPCHK(p.g, hipEventSynchronize(ws->ev[(d.k + 1) & 1]));
        }
        if (!reported()) d.status = st;
        return drive_end(d, block);
    }
    int rc = drive_enqueue(d);
    return rc == GG_OK ? 0 : rc;
}

// Blocking form: run the state machine to the end.
int plan_drive(Plan& p, long long r0, int stamp_base, int tag, long long* r_end) {
    Drive d;
    d.p = p;
    int rc = drive_start(d, r0, stamp_base, tag);
    while (rc == GG_OK) {
        rc = drive_step(d, true);
        if (rc == 1) break;
    }
    *r_end = d.r;
    if (rc < 0) return rc;
    return d.status;
}

void record_last(Plan& p, int status, long long rounds) {
    gg_ws ws = p.ws;
    ws->rounds = (int)rounds;
    ws->last_stream = p.s;
    ws->used = true;
    ws->last = gg_stats{};
    ws->last.algo = p.algo;
    ws->last.mode = p.o.mode;
    ws->last.sched = p.o.sched;
    ws->last.mapping = p.edge ? 0 : p.o.mapping;
    ws->last.status = status;
    ws->last.grid_blocks = p.g_round;
    ws->last.block_threads = kBlock;
}

int run_multi(gg_graph g, gg_ws ws, int algo, int source, const int* sources_dev, int nsrc,
              const gg_opts* opts, int* out, void* stream) {
    Plan p;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = plan_make(g, ws, algo, source, sources_dev, nsrc, opts, out, s, &p);
    if (rc != GG_OK) return rc;
    ws = p.ws;
    WsClaim claim(ws);
    if (!claim.held()) return GG_EBUSY;
    // a workspace serves one traversal at a time: order after its last one
    if (ws->used && ws->last_stream != s) HIPCHK(g, hipStreamWaitEvent(s, ws->finished, 0));
    p.prof = (p.o.flags & GG_OPT_PROFILE) != 0;
    ws->profiled = p.prof;
    ws->nlaunch = 0;
    hipError_t e;
    const int base = reserve_stamps(ws, s, (long long)g->n + 3, &e);
    HIPCHK(g, e);
    p.R.epoch = base;
    HIPCHK(g, plan_init(p));
    long long r_end = 0;
    const int status = plan_drive(p, 0, base, base, &r_end);
    if (status != GG_OK && status != GG_EITER && status != GG_ETIMEOUT) return status;
    // stamps of later traversals start after every round used here
    ws->epoch = (int)std::min<long long>((long long)base + r_end + 1, 1LL << 30);
    HIPCHK(g, hipEventRecord(ws->finished, s));
    record_last(p, status, r_end);
    return status;
}

}  // namespace gg

namespace {

int run(gg_graph g, gg_ws ws, int algo, int source, const gg_opts* opts, int* out, void* stream) {
    return run_multi(g, ws, algo, source, nullptr, 0, opts, out, stream);
}

}  // namespace

extern "C" {

int32_t gg_version(void) { return kVersion; }

const char* gg_status_str(int32_t status) {
    switch (status) {
        case GG_OK: return "GG_OK";
        case GG_EINVAL: return "GG_EINVAL";
        case GG_ENOMEM: return "GG_ENOMEM";
        case GG_EHIP: return "GG_EHIP";
        case GG_EBUSY: return "GG_EBUSY";
        case GG_ENOTSUP: return "GG_ENOTSUP";
        case GG_ETIMEOUT: return "GG_ETIMEOUT";
        case GG_EITER: return "GG_EITER";
        default: return "GG_UNKNOWN";
    }
}

int gg_graph_upload(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                    const int32_t* w, uint32_t flags, void* stream, gg_graph* out) {
    if (!out) return GG_EINVAL;
    *out = nullptr;
    if (n < 1 || m < 0 || m >= (1LL << 31) || !row_ptr || (m > 0 && !col)) return GG_EINVAL;
    const bool on_dev = flags & GG_INPUT_ON_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // host copy of the row offsets (needed for validation and heavy chunks)
    std::vector<int> hrow((size_t)n + 1);
    if (on_dev) {
        if (hipMemcpy(hrow.data(), row_ptr, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return GG_EHIP;
    } else {
        std::memcpy(hrow.data(), row_ptr, sizeof(int) * ((size_t)n + 1));
    }
    if (hrow[0] != 0 || hrow[n] != m) return GG_EINVAL;
    int max_deg = 0, argmax_deg = 0;
    for (int v = 0; v < n; ++v) {
        if (hrow[v + 1] < hrow[v]) return GG_EINVAL;
        if (hrow[v + 1] - hrow[v] > max_deg) {
            max_deg = hrow[v + 1] - hrow[v];
            argmax_deg = v;
        }
    }
    // host input: checked on the host (before any device work), in parallel
    HostCheck hc;
    if (!on_dev && m > 0) {
        hc = check_host(col, w, m, n);
        if (!hc.ok) return GG_EINVAL;
    }
    gg_graph g = new (std::nothrow) gg_graph_s();
    if (!g) return GG_ENOMEM;
    g->n = n;
    g->m = m;
    g->max_deg = max_deg;
    g->argmax_deg = argmax_deg;
    g->heavy = (double)max_deg >= 128.0 * ((double)m / (double)n) && m > 0 ? kHeavySkewed
                                                                            : kHeavyUniform;
    g->weighted = w != nullptr;
    if (!on_dev && w && m > 0) {
        g->max_w = hc.max_w;
        g->avg_w = (double)hc.wsum / (double)m;
    }
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    int* tmp = nullptr;  // in-degrees / fill cursors, and the check's statistics
    auto bail = [&](int code) {
        (void)hipStreamSynchronize(s);
        dfree(tmp);
        free_graph_arrays(g);
        delete g;
        return code;
    };
    auto grid = [&](long long units) {
        return (int)std::max(1LL, std::min<long long>(units, device().max_blocks));
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(&g->row, (size_t)n + 1);
    if (e == hipSuccess) e = dalloc(&g->col, (size_t)m);
    if (e == hipSuccess && w) e = dalloc(&g->w, (size_t)m);
    if (e == hipSuccess) e = dalloc(&g->src, (size_t)m);
    if (e == hipSuccess) e = dalloc(&tmp, (size_t)n + 8);
    if (e == hipSuccess) e = hipMemcpyAsync(g->row, hrow.data(), sizeof(int) * ((size_t)n + 1),
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess && m) e = hipMemcpyAsync(g->col, col, sizeof(int) * m, kind, s);
    if (e == hipSuccess && m && w) e = hipMemcpyAsync(g->w, w, sizeof(int) * m, kind, s);
    if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP);
    // device input: column range, weight sign, largest weight and weight
    // sum, checked on the device
    if (on_dev && m > 0) {
        int st[8] = {INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN, 0, 0, 0, 0};
        unsigned long long* dsum = reinterpret_cast<unsigned long long*>(tmp + 4);
        e = hipMemcpyAsync(tmp, st, sizeof(st), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_check(g->col, g->w, (int)m, tmp, dsum, grid((m + 4095) / 4096), s);
        if (e == hipSuccess) e = hipMemcpyAsync(st, tmp, sizeof(st), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(GG_EHIP);
        if (st[0] < 0 || st[1] >= n) return bail(GG_EINVAL);
        if (w) {
            if (st[2] < 0) return bail(GG_EINVAL);
            unsigned long long sum = 0;
            std::memcpy(&sum, st + 4, sizeof(sum));
            g->max_w = st[3];
            g->avg_w = (double)sum / (double)m;
        }
    }
    // hottest vertices first: on request, or on a skewed graph large enough
    // that its values do not fit in the dies' caches anyway
    std::vector<int> hin;
    const bool renumber = !(flags & GG_KEEP_ORDER) && m > 0 && n > 1 &&
                          ((flags & GG_RENUMBER) ||
                           (g->heavy == kHeavySkewed && m >= kPartMinEdges));
    if (renumber) {
        const int rc = renumber_graph(g, hrow, hin, tmp, s);
        if (rc != GG_OK) return bail(rc);
    }
    e = launch_fill_src(g->row, n, (int)m, g->src, grid((m + 4095) / 4096), kBlock, s);
    if (e != hipSuccess) return bail(GG_EHIP);
    // in-degrees, counted once for the head-partitioned edge list, the
    // both-directions CSR and the in-edge CSR
    const bool sym_build = (flags & GG_SYMMETRIZE) && !(flags & GG_SYMMETRIC);
    if (m > 0 && !renumber && (m >= kPartMinEdges || sym_build || (flags & GG_TRANSPOSE))) {
        hin.resize((size_t)n);
        e = hipMemsetAsync(tmp, 0, sizeof(int) * n, s);
        if (e == hipSuccess)
            e = launch_count_in(g->col, (int)m, tmp, grid((m + kBlock - 1) / kBlock), kBlock, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hin.data(), tmp, sizeof(int) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(GG_EHIP);
    }
    if (m >= kPartMinEdges) {
        const int rc = build_parts(g, hin, s);
        if (rc != GG_OK) return bail(rc);
    }
    std::vector<int2> hch = build_chunks(hrow, n, g->heavy, g->chunk);
    g->n_hchunks = (int)hch.size();
    if (!hch.empty()) {
        e = dalloc(&g->hchunks, hch.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->hchunks, hch.data(), sizeof(int2) * hch.size(),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(GG_EHIP);
    }
    if (flags & GG_SYMMETRIC) {
        g->symmetric = true;
        g->has_sym = true;
        g->srow = g->row;
        g->scol = g->col;
        g->ssrc = g->src;
        g->ms = m;
        g->n_shchunks = g->n_hchunks;
        if (g->n_hchunks) {
            e = dalloc(&g->shchunks, hch.size());
            if (e == hipSuccess)
                e = hipMemcpyAsync(g->shchunks, hch.data(), sizeof(int2) * hch.size(),
                                   hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return bail(GG_EHIP);
        }
    } else if (flags & GG_SYMMETRIZE) {
        const long long ms = 2 * m;
        if (ms >= (1LL << 31)) return bail(GG_EINVAL);
        std::vector<int> hsrow((size_t)n + 1);
        hsrow[0] = 0;
        for (int v = 0; v < n; ++v)
            hsrow[v + 1] = hsrow[v] + (hrow[v + 1] - hrow[v]) + (m > 0 ? hin[v] : 0);
        if (e == hipSuccess) e = dalloc(&g->srow, (size_t)n + 1);
        if (e == hipSuccess) e = dalloc(&g->scol, (size_t)ms);
        if (e == hipSuccess) e = dalloc(&g->ssrc, (size_t)ms);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->srow, hsrow.data(), sizeof(int) * ((size_t)n + 1),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(tmp, 0, sizeof(int) * n, s);
        if (e == hipSuccess && m)
            e = launch_sym_fill(g->row, g->col, g->src, n, (int)m, g->srow, tmp, g->scol,
                                grid((m + kBlock - 1) / kBlock), kBlock, s);
        if (e == hipSuccess)
            e = launch_fill_src(g->srow, n, (int)ms, g->ssrc, grid((ms + 4095) / 4096), kBlock, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP);
        g->has_sym = true;
        g->ms = ms;
        std::vector<int2> sch = build_chunks(hsrow, n, g->heavy, g->chunk);
        g->n_shchunks = (int)sch.size();
        if (!sch.empty()) {
            e = dalloc(&g->shchunks, sch.size());
            if (e == hipSuccess)
                e = hipMemcpyAsync(g->shchunks, sch.data(), sizeof(int2) * sch.size(),
                                   hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return bail(GG_EHIP);
        }
    }
    if ((flags & GG_TRANSPOSE) && m > 0) {
        // weighted in-edge CSR: prefix sums of the in-degrees on the host,
        // then every edge placed in its head's row
        std::vector<int> htrow((size_t)n + 1);
        htrow[0] = 0;
        for (int v = 0; v < n; ++v) htrow[v + 1] = htrow[v] + hin[v];
        if (e == hipSuccess) e = dalloc(&g->trow, (size_t)n + 1);
        if (e == hipSuccess) e = dalloc(&g->tcol, (size_t)m);
        if (e == hipSuccess) e = dalloc(&g->tw, (size_t)m);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->trow, htrow.data(), sizeof(int) * ((size_t)n + 1),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(tmp, 0, sizeof(int) * n, s);
        if (e == hipSuccess)
            e = launch_t_fill(g->col, g->w, g->src, (int)m, g->trow, tmp, g->tcol, g->tw,
                              grid((m + kBlock - 1) / kBlock), kBlock, s);
        std::vector<int2> tch;
        if (e == hipSuccess) tch = build_chunks(htrow, n, g->heavy, g->chunk);
        g->n_tchunks = (int)tch.size();
        if (e == hipSuccess && !tch.empty()) {
            e = dalloc(&g->tchunks, tch.size());
            if (e == hipSuccess)
                e = hipMemcpyAsync(g->tchunks, tch.data(), sizeof(int2) * tch.size(),
                                   hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP);
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(GG_EHIP);
    dfree(tmp);
    int rc = make_ws(g, &g->ws0);
    if (rc != GG_OK) return bail(rc);
    g->ws0->is_default = true;
    *out = g;
    return GG_OK;
}

int gg_graph_free(gg_graph g) {
    if (!g) return GG_EINVAL;
    if (g->n_ws > 0 || g->n_async.load() > 0) return GG_EBUSY;
    (void)hipDeviceSynchronize();
    free_ws_arrays(g->ws0);
    delete g->ws0;
    free_graph_arrays(g);
    delete g;
    return GG_OK;
}

int gg_graph_info(gg_graph g, int32_t* n, int64_t* m, int32_t* max_out_degree,
                  int32_t* has_weights, int32_t* has_sym) {
    if (!g) return GG_EINVAL;
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_out_degree) *max_out_degree = g->max_deg;
    if (has_weights) *has_weights = g->weighted;
    if (has_sym) *has_sym = g->has_sym;
    return GG_OK;
}

int gg_graph_error(gg_graph g) { return g ? g->err : GG_EINVAL; }

int gg_graph_order(gg_graph g, int32_t* renumbered) {
    if (!g || !renumbered) return GG_EINVAL;
    *renumbered = g->renumbered ? 1 : 0;
    return GG_OK;
}

int gg_ws_create(gg_graph g, gg_ws* out) {
    if (!g || !out) return GG_EINVAL;
    gg_ws_s* ws = nullptr;
    int rc = make_ws(g, &ws);
    if (rc != GG_OK) return rc;
    g->n_ws++;
    *out = ws;
    return GG_OK;
}

int gg_ws_free(gg_ws ws) {
    if (!ws || ws->is_default) return GG_EINVAL;
    if (ws->busy.load()) return GG_EBUSY;
    if (ws->used) (void)hipEventSynchronize(ws->finished);
    ws->owner->n_ws--;
    free_ws_arrays(ws);
    delete ws;
    return GG_OK;
}

int gg_sssp_ex(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
               void* stream) {
    return run(g, ws, GG_ALGO_SSSP, source, opts, dist_out_dev, stream);
}

int gg_bfs_ex(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
              void* stream) {
    return run(g, ws, GG_ALGO_BFS, source, opts, dist_out_dev, stream);
}

int gg_cc_ex(gg_graph g, gg_ws ws, const gg_opts* opts, int32_t* label_out_dev, void* stream) {
    return run(g, ws, GG_ALGO_CC, 0, opts, label_out_dev, stream);
}

int gg_sssp(gg_graph g, int32_t source, int32_t mode, int32_t sched, int32_t* dist_out_dev,
            void* stream) {
    gg_opts o{};
    o.mode = mode;
    o.sched = sched;
    return run(g, nullptr, GG_ALGO_SSSP, source, &o, dist_out_dev, stream);
}

int gg_bfs(gg_graph g, int32_t source, int32_t mode, int32_t sched, int32_t* dist_out_dev,
           void* stream) {
    gg_opts o{};
    o.mode = mode;
    o.sched = sched;
    return run(g, nullptr, GG_ALGO_BFS, source, &o, dist_out_dev, stream);
}

int gg_cc(gg_graph g, int32_t mode, int32_t sched, int32_t* label_out_dev, void* stream) {
    gg_opts o{};
    o.mode = mode;
    o.sched = sched;
    return run(g, nullptr, GG_ALGO_CC, 0, &o, label_out_dev, stream);
}

int gg_last_stats(gg_graph g, gg_ws ws, gg_stats* out) {
    if (!g || !out) return GG_EINVAL;
    if (!ws) ws = g->ws0;
    if (ws->owner != g) return GG_EINVAL;
    if (ws->busy.load()) return GG_EBUSY;
    if (!ws->used) {
        *out = gg_stats{};
        return GG_OK;
    }
    HIPCHK(g, hipEventSynchronize(ws->finished));
    Ctl c;
    std::vector<Stat> st((size_t)kKinds * kMaxStatBlocks);
    HIPCHK(g, hipMemcpy(&c, ws->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    HIPCHK(g, hipMemcpy(st.data(), ws->dev.stat, sizeof(Stat) * st.size(),
                        hipMemcpyDeviceToHost));
    gg_stats s = ws->last;
    s.iterations = c.done ? c.iters : -1;
    for (const Stat& x : st) {
        s.edges_processed += x.edges;
        s.vertices_processed += x.verts;
        s.updates += x.updates;
        s.pushes += x.pushes;
    }
    *out = s;
    return s.status;
}

int gg_last_profile(gg_graph g, gg_ws ws, gg_profile* out) {
    if (!g || !out) return GG_EINVAL;
    if (!ws) ws = g->ws0;
    if (ws->owner != g) return GG_EINVAL;
    if (ws->busy.load()) return GG_EBUSY;
    *out = gg_profile{};
    if (!ws->used || !ws->profiled) return GG_OK;
    HIPCHK(g, hipEventSynchronize(ws->finished));
    std::vector<Stat> st((size_t)kKinds * kMaxStatBlocks);
    HIPCHK(g, hipMemcpy(st.data(), ws->dev.stat, sizeof(Stat) * st.size(),
                        hipMemcpyDeviceToHost));
    out->profiled = 1;
    out->rounds = ws->rounds;
    if (g_time_ref && ws->nlaunch > 0) {
        float b = 0.f, e = 0.f;
        HIPCHK(g, hipEventElapsedTime(&b, g_time_ref, ws->pev[0]));
        HIPCHK(g, hipEventElapsedTime(&e, g_time_ref, ws->pev[2 * ws->nlaunch - 1]));
        out->begin_ms = b;
        out->end_ms = e;
    }
    for (int i = 0; i < ws->nlaunch; ++i) {
        float ms = 0.f;
        HIPCHK(g, hipEventElapsedTime(&ms, ws->pev[2 * i], ws->pev[2 * i + 1]));
        gg_kind_profile& k = out->kind[ws->pkind[i]];
        k.launches++;
        k.total_ms += ms;
    }
    for (int kind = 0; kind < kKinds; ++kind)
        for (int b = 0; b < kMaxStatBlocks; ++b) {
            const Stat& x = st[(size_t)kind * kMaxStatBlocks + b];
            out->kind[kind].edges_processed += x.edges;
            out->kind[kind].vertices_processed += x.verts;
            out->kind[kind].updates += x.updates;
            out->kind[kind].pushes += x.pushes;
            out->kind[kind].swept_edges += x.swept;
        }
    return GG_OK;
}

int gg_graph_probe(gg_graph g, void* stream) {
    if (!g) return GG_EINVAL;
    int* dist = nullptr;
    HIPCHK(g, dalloc(&dist, (size_t)g->n));
    gg_opts o{};
    o.mode = GG_VERTEX;
    o.sched = GG_ASYNC;
    o.mapping = GG_MAP_BALANCED;
    int rc = run(g, nullptr, GG_ALGO_BFS, g->argmax_deg, &o, dist, stream);
    gg_stats st{};
    if (rc == GG_OK) rc = gg_last_stats(g, nullptr, &st);
    (void)hipFree(dist);  // waits for the traversal; a failure of it shows in rc
    if (rc != GG_OK) return rc;
    g->levels = st.iterations;
    return GG_OK;
}

int gg_graph_class(gg_graph g, int32_t* size_class, int32_t* skew_class, int32_t* depth_class) {
    if (!g) return GG_EINVAL;
    return gg_class_of(g->m, g->n, g->max_deg, g->levels, size_class, skew_class, depth_class);
}

int gg_resolve(gg_graph g, int32_t algo, const gg_opts* in, gg_opts* out) {
    if (!g || !out || algo < 0 || algo > 2) return GG_EINVAL;
    resolve(g, algo, in, out);
    return GG_OK;
}

}  // extern "C"
