// gg_batch.hip -- batched SSSP/BFS over many independent instances
// (declared in include/gg.h).
//
// Instances of one algorithm and one graph class are concatenated into a
// single graph: instance j's vertex v becomes base_j + v and its edges keep
// their heads inside the instance, so every instance is a set of components
// of its own.  One multi-source traversal of the group (one source per
// instance) then computes each instance exactly as a separate call would.
// The group is a regular uploaded graph with its own workspace and stream;
// after its first (eager) run its launch sequence -- init, seed and a fixed
// number of rounds -- is captured in a HIP graph and replayed by later runs.

#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "gg_runtime.h"

using namespace gg;

namespace {

struct Group {
    int algo = 0;
    std::vector<int> members;  // instance indices, in order
    std::vector<long long> vbase;
    long long n = 0, m = 0;
    long long out_off = 0;     // first output slot of the group
    gg_graph g = nullptr;
    int* sources = nullptr;    // device, concatenated ids
    int nsrc = 0;
    gg_opts opts{};            // variant the group runs
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int* h_ctl = nullptr;      // pinned copy of (done, rounds) after a replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int* graph_out = nullptr;  // output pointer baked into the captured graph
    int r_cap = 0;
    int last_rounds = 0;
};

}  // namespace

struct gg_batch_s {
    std::vector<Group> groups;
    std::vector<long long> v_off;
    long long total_n = 0, total_m = 0;
    uint32_t flags = 0;
    hipEvent_t start = nullptr;
};

namespace {

bool valid_instance(const gg_instance& x, int* max_deg) {
    if ((x.algo != GG_ALGO_SSSP && x.algo != GG_ALGO_BFS) || x.n < 1 || x.m < 0 ||
        x.m >= (1LL << 31) || !x.row_ptr || (x.m > 0 && !x.col) || x.source < 0 ||
        x.source >= x.n || (x.algo == GG_ALGO_SSSP && x.m > 0 && !x.w))
        return false;
    if (x.row_ptr[0] != 0 || x.row_ptr[x.n] != x.m) return false;
    int md = 0;
    for (int v = 0; v < x.n; ++v) {
        const int d = x.row_ptr[v + 1] - x.row_ptr[v];
        if (d < 0) return false;
        md = d > md ? d : md;
    }
    *max_deg = md;
    return true;
}

void destroy_group(Group& G) {
    if (G.stream) (void)hipStreamSynchronize(G.stream);
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    if (G.g) gg_graph_free(G.g);
    if (G.sources) (void)hipFree(G.sources);
    if (G.h_ctl) (void)hipHostFree(G.h_ctl);
    if (G.done) (void)hipEventDestroy(G.done);
    if (G.stream) (void)hipStreamDestroy(G.stream);
    G = Group{};
}

// Capture init, seed and G.r_cap rounds of the group into a HIP graph.
int capture(Group& G, int* out) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    G.exec = nullptr;
    G.graph = nullptr;
    Plan p;
    int rc = plan_make(G.g, nullptr, G.algo, 0, G.sources, G.nsrc, &G.opts, out, G.stream, &p);
    if (rc != GG_OK) return rc;
    hipError_t e;
    // the tag is reserved before the capture begins; every replay uses it
    const int base = reserve_stamps(p.ws, G.stream, (long long)G.r_cap + 1, &e);
    if (e != hipSuccess) return GG_EHIP;
    p.R.epoch = base;
    if (hipStreamBeginCapture(G.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return GG_EHIP;
    e = plan_init(p);
    for (int r = 0; r < G.r_cap && e == hipSuccess; ++r) e = plan_round(p, r);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(G.stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return GG_EHIP;
    }
    if (hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return GG_EHIP;
    }
    G.graph = graph;
    G.graph_out = out;
    return GG_OK;
}

}  // namespace

extern "C" {

int gg_batch_create(const gg_instance* inst, int32_t count, uint32_t flags, void* stream,
                    gg_batch* out) {
    if (!out) return GG_EINVAL;
    *out = nullptr;
    if (!inst || count < 1) return GG_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // group key: algorithm and graph class (size, skew) of the instance
    std::map<std::tuple<int, int, int>, std::vector<int>> keys;
    for (int i = 0; i < count; ++i) {
        int md = 0;
        if (!valid_instance(inst[i], &md)) return GG_EINVAL;
        int32_t sc = 0, kc = 0, dc = 0;
        gg_class_of(inst[i].m, inst[i].n, md, -1, &sc, &kc, &dc);
        if (flags & GG_BATCH_ONE_GROUP) sc = kc = 0;
        keys[std::make_tuple(inst[i].algo, sc, kc)].push_back(i);
    }
    gg_batch b = new (std::nothrow) gg_batch_s();
    if (!b) return GG_ENOMEM;
    b->flags = flags;
    b->v_off.assign(count, 0);
    auto bail = [&](int code) {
        for (Group& G : b->groups) destroy_group(G);
        if (b->start) (void)hipEventDestroy(b->start);
        delete b;
        return code;
    };
    if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess)
        return bail(GG_EHIP);
    long long out_off = 0;
    for (auto& kv : keys) {
        b->groups.emplace_back();
        Group& G = b->groups.back();
        G.algo = std::get<0>(kv.first);
        G.members = kv.second;
        for (int i : G.members) {
            G.vbase.push_back(G.n);
            G.n += inst[i].n;
            G.m += inst[i].m;
        }
        if (G.n >= (1LL << 31) || G.m >= (1LL << 31)) return bail(GG_EINVAL);
        const bool weighted = G.algo == GG_ALGO_SSSP;
        std::vector<int> row((size_t)G.n + 1), col((size_t)std::max(G.m, 1LL));
        std::vector<int> w(weighted ? (size_t)std::max(G.m, 1LL) : 0);
        std::vector<int> src;
        long long eb = 0;
        for (size_t k = 0; k < G.members.size(); ++k) {
            const gg_instance& x = inst[G.members[k]];
            const int vb = (int)G.vbase[k];
            for (int v = 0; v < x.n; ++v) row[vb + v] = (int)(eb + x.row_ptr[v]);
            for (long long e = 0; e < x.m; ++e) col[eb + e] = vb + x.col[e];
            if (weighted && x.m) std::memcpy(&w[eb], x.w, sizeof(int) * (size_t)x.m);
            src.push_back(vb + x.source);
            b->v_off[G.members[k]] = out_off + vb;
            eb += x.m;
        }
        row[G.n] = (int)eb;
        G.out_off = out_off;
        out_off += G.n;
        b->total_m += G.m;
        // the group's traversal starts from a device list of caller ids:
        // kept in the caller's vertex order
        int rc = gg_graph_upload((int)G.n, G.m, row.data(), col.data(),
                                 weighted ? w.data() : nullptr, GG_KEEP_ORDER, stream, &G.g);
        if (rc != GG_OK) return bail(rc);
        G.nsrc = (int)src.size();
        if (dalloc(&G.sources, src.size()) != hipSuccess ||
            hipMemcpyAsync(G.sources, src.data(), sizeof(int) * src.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(GG_EHIP);
        if (hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&G.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&G.h_ctl), 2 * sizeof(int)) != hipSuccess)
            return bail(GG_EHIP);
        gg_resolve(G.g, G.algo, nullptr, &G.opts);
        // The table's choice is measured on single-source traversals.  A
        // group is one traversal from hundreds of sources over as many small
        // components: near-far rounds then follow the component that needs
        // the most buckets, while the repeated hub expansions the buckets
        // save belong to large skewed graphs (measured on 512 R-MAT
        // instances of scales 10-18: near-far with long-row deferral 18.4 ms
        // per run, the plain worklist 14.0 ms).  Groups run the worklist.
        if (G.opts.sched == GG_NEARFAR) {
            G.opts.sched = GG_ASYNC;
            G.opts.delta = 0;
            G.opts.far_degree = 0;
            G.opts.hops = 0;
        }
    }
    b->total_n = out_off;
    *out = b;
    return GG_OK;
}

int gg_batch_run(gg_batch b, int32_t* out_dev, void* stream) {
    if (!b || !out_dev) return GG_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool graphs = !(b->flags & GG_BATCH_NO_GRAPH);
    if (hipEventRecord(b->start, s) != hipSuccess) return GG_EHIP;
    std::vector<char> replayed(b->groups.size(), 0);
    int status = GG_OK;
    // launch every group: replays go out at once; a group without a graph
    // (first run, other output, or graphs off) runs eagerly and is captured
    for (size_t i = 0; i < b->groups.size(); ++i) {
        Group& G = b->groups[i];
        int* out = out_dev + G.out_off;
        if (hipStreamWaitEvent(G.stream, b->start, 0) != hipSuccess) return GG_EHIP;
        if (graphs && G.exec && G.graph_out == out) {
            Ctl* ctl = G.g->ws0->dev.ctl;
            if (hipGraphLaunch(G.exec, G.stream) != hipSuccess ||
                hipMemcpyAsync(G.h_ctl, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, G.stream) !=
                    hipSuccess ||
                hipEventRecord(G.done, G.stream) != hipSuccess)
                return GG_EHIP;
            replayed[i] = 1;
            continue;
        }
        int rc = run_multi(G.g, nullptr, G.algo, 0, G.sources, G.nsrc, &G.opts, out, G.stream);
        if (rc != GG_OK) status = rc;
        gg_stats st{};
        if (gg_last_stats(G.g, nullptr, &st) == GG_OK) G.last_rounds = st.iterations;
        if (rc == GG_OK && graphs) {
            // room for the rounds just used and a margin (asynchronous rounds
            // vary a little from run to run)
            G.r_cap = G.last_rounds + G.last_rounds / 4 + 2;
            rc = capture(G, out);
            if (rc != GG_OK) status = rc;
        }
        if (hipEventRecord(G.done, G.stream) != hipSuccess) return GG_EHIP;
    }
    // replays that stopped short of the end continue eagerly
    for (size_t i = 0; i < b->groups.size(); ++i) {
        if (!replayed[i]) continue;
        Group& G = b->groups[i];
        if (hipEventSynchronize(G.done) != hipSuccess) return GG_EHIP;
        if (G.h_ctl[0]) {
            G.last_rounds = G.h_ctl[1];
            continue;
        }
        Plan p;
        int rc = plan_make(G.g, nullptr, G.algo, 0, G.sources, G.nsrc, &G.opts,
                           out_dev + G.out_off, G.stream, &p);
        hipError_t e = hipSuccess;
        const int base = rc == GG_OK ? reserve_stamps(p.ws, G.stream, (long long)G.n + 3, &e) : 0;
        if (rc != GG_OK || e != hipSuccess) return rc != GG_OK ? rc : GG_EHIP;
        p.R.epoch = base;
        long long r_end = 0;
        rc = plan_drive(p, G.r_cap, base, base, &r_end);
        p.ws->epoch = (int)std::min<long long>((long long)base + r_end + 1, 1LL << 30);
        record_last(p, rc, r_end);
        if (rc != GG_OK) status = rc;
        G.last_rounds = (int)r_end;
        G.r_cap = (int)(r_end + r_end / 4 + 2);  // the next run recaptures
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
        if (hipEventRecord(G.done, G.stream) != hipSuccess) return GG_EHIP;
    }
    for (Group& G : b->groups) {
        gg_ws ws = G.g->ws0;
        ws->last_stream = G.stream;
        ws->used = true;
        if (hipEventRecord(ws->finished, G.stream) != hipSuccess ||
            hipStreamWaitEvent(s, G.done, 0) != hipSuccess)
            return GG_EHIP;
    }
    return status;
}

int gg_batch_offsets(gg_batch b, int64_t* v_off) {
    if (!b || !v_off) return GG_EINVAL;
    for (size_t i = 0; i < b->v_off.size(); ++i) v_off[i] = b->v_off[i];
    return GG_OK;
}

int gg_batch_info(gg_batch b, int32_t* groups, int64_t* total_n, int64_t* total_m) {
    if (!b) return GG_EINVAL;
    if (groups) *groups = (int32_t)b->groups.size();
    if (total_n) *total_n = b->total_n;
    if (total_m) *total_m = b->total_m;
    return GG_OK;
}

int gg_batch_group(gg_batch b, int32_t g, int32_t* algo, int32_t* instances, int64_t* n,
                   int64_t* m, int32_t* mode, int32_t* sched, int32_t* mapping,
                   int32_t* captured_rounds, int32_t* last_rounds) {
    if (!b || g < 0 || g >= (int32_t)b->groups.size()) return GG_EINVAL;
    const Group& G = b->groups[g];
    if (algo) *algo = G.algo;
    if (instances) *instances = (int32_t)G.members.size();
    if (n) *n = G.n;
    if (m) *m = G.m;
    if (mode) *mode = G.opts.mode;
    if (sched) *sched = G.opts.sched;
    if (mapping) *mapping = G.opts.mapping;
    if (captured_rounds) *captured_rounds = G.exec ? G.r_cap : 0;
    if (last_rounds) *last_rounds = G.last_rounds;
    return GG_OK;
}

int gg_batch_free(gg_batch b) {
    if (!b) return GG_EINVAL;
    for (Group& G : b->groups) destroy_group(G);
    if (b->start) (void)hipEventDestroy(b->start);
    delete b;
    return GG_OK;
}

}  // extern "C"
