// gg_serve.hip -- serving loop: SSSP/BFS queries admitted as they arrive and
// advanced together on a pool of streams (declared in include/gg.h).
//
// A query needs a workspace of its graph (per-query frontier flags,
// heavy-row bits, control block) and a stream.  Workspaces are pooled per graph and
// reused; the bytes of the workspaces held by queries in flight are bounded
// by the memory budget.  Admission is first-come first-served: when the
// head of the queue does not fit (no slot, or its state would exceed the
// budget), later queries wait behind it.  A driver thread of the server
// admits queries and advances each one in flight by a batch of rounds as
// soon as its previous batch completes (non-blocking event queries), so the
// kernels of different queries overlap on the device and no caller thread
// sits on the path between two batches; gg_server_poll only hands out the
// finished queries.

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <new>
#include <thread>
#include <vector>

#include "gg_runtime.h"

using namespace gg;

namespace {

struct SGraph {
    gg_graph g = nullptr;
    int in_use = 0;            // queued + in flight
    bool retiring = false;
    std::vector<gg_ws> pool;   // idle workspaces
    std::vector<gg_ws> all;
    long long ws_bytes = 0;    // bytes of one workspace
};

struct Query {
    long long id = 0;
    int graph_id = 0, algo = 0, source = 0;
    int* out = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    double t_submit = 0, t_admit = 0, t_done = 0;
    gg_ws ws = nullptr;
    int stream = -1;
    Drive d;
};

long long ws_bytes_of(gg_graph g) {
    const long long ntiles = (g->n + 63) / 64;
    const long long vbytes = ((ntiles + 63) / 64) * 64 * 64;
    const long long tbytes = ((ntiles + 63) / 64) * 64;
    const long long hwords = (g->n + 31) / 32;
    const long long renum = g->renumbered ? 8LL * g->n : 0;  // values and minima
    return 2 * (vbytes + tbytes) + 2 * 4LL * hwords + renum + (long long)sizeof(Ctl) +
           (long long)sizeof(Stat) * kKinds * kMaxStatBlocks + 4LL * 3 * 2 * kMaxStatBlocks;
}

}  // namespace

struct gg_server_s {
    std::mutex mu;  // everything below (callers vs the driver thread)
    std::condition_variable wake;  // work arrived, or stop
    std::thread driver;
    bool stop = false;
    int device = 0;
    std::map<int, SGraph> graphs;
    int next_graph = 0;
    long long next_query = 0;
    std::deque<Query*> queue;
    std::vector<Query*> active;
    std::deque<gg_query_result> finished;  // not yet handed out by poll
    std::vector<hipStream_t> streams;
    std::vector<char> stream_busy;
    std::vector<hipEvent_t> spare_events;  // for Query::ready
    int slots = 0;
    long long budget = 0, used = 0;
    long long alloc = 0;  // bytes of every workspace allocated (pooled or in flight)
    std::chrono::steady_clock::time_point t0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void free_graph_entry(SGraph& G) {
    if (G.g) {
        (void)hipDeviceSynchronize();
        for (gg_ws w : G.all) gg_ws_free(w);
        gg_graph_free(G.g);
    }
    G = SGraph{};
}

void release_event(gg_server s, Query* q) {
    if (q->ready) s->spare_events.push_back(q->ready);
    q->ready = nullptr;
}

// Free the idle pooled workspaces of graphs other than `keep` until a new
// workspace of `need` bytes fits the budget (freeing device memory waits for
// the device, so this runs only when the budget forces it).
void trim_pools(gg_server s, int keep, long long need) {
    for (auto& kv : s->graphs) {
        if (s->alloc + need <= s->budget) return;
        if (kv.first == keep) continue;
        SGraph& G = kv.second;
        while (!G.pool.empty() && s->alloc + need > s->budget) {
            gg_ws w = G.pool.back();
            G.pool.pop_back();
            G.all.erase(std::find(G.all.begin(), G.all.end(), w));
            gg_ws_free(w);
            s->alloc -= G.ws_bytes;
        }
    }
}

// Retired graphs with nothing queued or in flight are freed while the
// server has no query in flight (freeing device memory waits for the whole
// device, which then costs no query anything).
void reap_retired(gg_server s) {
    if (!s->active.empty()) return;
    for (auto it = s->graphs.begin(); it != s->graphs.end();) {
        SGraph& G = it->second;
        if (G.retiring && G.in_use == 0) {
            s->alloc -= (long long)G.all.size() * G.ws_bytes;
            free_graph_entry(G);
            it = s->graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// Start a query on a free stream with a workspace of its graph.
int admit(gg_server s, Query* q, SGraph& G) {
    int si = -1;
    for (int i = 0; i < (int)s->streams.size(); ++i)
        if (!s->stream_busy[i]) {
            si = i;
            break;
        }
    if (si < 0) return GG_EBUSY;
    gg_ws ws = nullptr;
    if (!G.pool.empty()) {
        ws = G.pool.back();
        G.pool.pop_back();
    } else {
        if (s->budget > 0) trim_pools(s, q->graph_id, G.ws_bytes);
        int rc = gg_ws_create(G.g, &ws);
        if (rc != GG_OK) return rc;
        G.all.push_back(ws);
        s->alloc += G.ws_bytes;
    }
    hipStream_t st = s->streams[si];
    Plan& p = q->d.p;
    int rc = plan_make(G.g, ws, q->algo, q->source, nullptr, 0, nullptr, q->out, st, &p);
    // after the caller's work on the output before submission, and after the
    // workspace's last query
    if (rc == GG_OK && q->ready)
        rc = hipStreamWaitEvent(st, q->ready, 0) == hipSuccess ? GG_OK : GG_EHIP;
    if (rc == GG_OK && ws->used && ws->last_stream != st)
        rc = hipStreamWaitEvent(st, ws->finished, 0) == hipSuccess ? GG_OK : GG_EHIP;
    hipError_t e = hipSuccess;
    const int base = rc == GG_OK ? reserve_stamps(ws, st, (long long)G.g->n + 3, &e) : 0;
    if (rc == GG_OK && e != hipSuccess) rc = GG_EHIP;
    if (rc == GG_OK) {
        p.R.epoch = base;
        if (plan_init(p) != hipSuccess) rc = GG_EHIP;
    }
    q->d.poll = true;
    if (rc == GG_OK) rc = drive_start(q->d, 0, base, base);
    if (rc != GG_OK) {
        // kernels may already be enqueued: the workspace's next query is
        // ordered after them
        (void)hipEventRecord(ws->finished, st);
        ws->last_stream = st;
        ws->used = true;
        G.pool.push_back(ws);
        return rc;
    }
    q->ws = ws;
    q->stream = si;
    s->stream_busy[si] = 1;
    return GG_OK;
}

// One pass of the driver with the lock held: admission (first come, first
// served, while a slot and the memory budget allow), then every query in
// flight advances by at most one batch.  Returns whether anything changed.
bool step_locked(gg_server s) {
    bool moved = false;
    while (!s->queue.empty() && (int)s->active.size() < s->slots) {
        Query* q = s->queue.front();
        SGraph& G = s->graphs[q->graph_id];
        if (s->budget > 0 && s->used + G.ws_bytes > s->budget && !s->active.empty()) break;
        int rc = admit(s, q, G);
        if (rc == GG_EBUSY) break;
        s->queue.pop_front();
        moved = true;
        q->t_admit = s->now();
        if (rc != GG_OK) {
            // failed to start: report at once
            q->t_done = q->t_admit;
            s->finished.push_back(gg_query_result{q->id, rc, 0, q->t_submit, q->t_admit, q->t_done});
            G.in_use--;
            release_event(s, q);
            delete q;
            continue;
        }
        s->used += G.ws_bytes;
        s->active.push_back(q);
    }
    for (size_t i = 0; i < s->active.size();) {
        Query* q = s->active[i];
        const long long r_before = q->d.r;
        const int rc = drive_step(q->d, false);
        if (rc == 0) {
            moved |= q->d.r != r_before;
            ++i;
            continue;
        }
        moved = true;
        q->t_done = s->now();
        const int status = rc < 0 ? rc : q->d.status;
        Plan& p = q->d.p;
        if (hipEventRecord(q->ws->finished, p.s) != hipSuccess && rc >= 0) {
            // keep going: the status of this query reports the failure
        }
        record_last(p, status, q->d.r);
        // stamps of the workspace's next query start after every round used
        q->ws->epoch = std::max(q->ws->epoch,
                                (int)std::min<long long>(q->d.stamp_base + q->d.r + 1, 1LL << 30));
        SGraph& G = s->graphs[q->graph_id];
        G.pool.push_back(q->ws);
        s->used -= G.ws_bytes;
        s->stream_busy[q->stream] = 0;
        s->finished.push_back(gg_query_result{q->id, status, (int32_t)q->d.r, q->t_submit,
                                              q->t_admit, q->t_done});
        G.in_use--;
        release_event(s, q);
        delete q;
        s->active[i] = s->active.back();
        s->active.pop_back();
    }
    reap_retired(s);
    return moved;
}

// The driver: sleeps while there is nothing to do; otherwise steps, and
// between steps that change nothing releases the lock and yields (a batch
// of rounds takes microseconds to milliseconds; polling keeps the gap
// between a batch's end and the next launch short).
void drive_loop(gg_server s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        if (s->queue.empty() && s->active.empty()) {
            reap_retired(s);
            s->wake.wait(lk);
            continue;
        }
        if (!step_locked(s)) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

int gg_server_create(int32_t slots, int64_t mem_budget_bytes, gg_server* out) {
    if (!out || slots < 1 || slots > 1024 || mem_budget_bytes < 0) return GG_EINVAL;
    gg_server s = new (std::nothrow) gg_server_s();
    if (!s) return GG_ENOMEM;
    s->slots = slots;
    s->budget = mem_budget_bytes;
    s->t0 = std::chrono::steady_clock::now();
    s->streams.assign(slots, nullptr);
    s->stream_busy.assign(slots, 0);
    bool ok = hipGetDevice(&s->device) == hipSuccess;
    for (int i = 0; ok && i < slots; ++i)
        ok = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        try {
            s->driver = std::thread(drive_loop, s);
        } catch (...) {
            ok = false;
        }
    }
    if (!ok) {
        for (hipStream_t st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        delete s;
        return GG_EHIP;
    }
    *out = s;
    return GG_OK;
}

int gg_server_add_graph(gg_server s, gg_graph g, int32_t* graph_id) {
    if (!s || !g || !graph_id) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int id = s->next_graph++;
    SGraph& G = s->graphs[id];
    G.g = g;
    G.ws_bytes = ws_bytes_of(g);
    *graph_id = id;
    return GG_OK;
}

int gg_server_remove_graph(gg_server s, int32_t graph_id) {
    if (!s) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->graphs.find(graph_id);
    if (it == s->graphs.end() || it->second.retiring) return GG_EINVAL;
    // no new submissions; the memory is released once its queries are done
    // and the server has nothing in flight (freeing device memory waits for
    // the whole device)
    it->second.retiring = true;
    s->wake.notify_one();
    return GG_OK;
}

int gg_server_submit(gg_server s, int32_t graph_id, int32_t algo, int32_t source,
                     int32_t* out_dev, void* stream, int64_t* query_id) {
    if (!s || !out_dev || (algo != GG_ALGO_SSSP && algo != GG_ALGO_BFS)) return GG_EINVAL;
    Query* q = new (std::nothrow) Query();
    if (!q) return GG_ENOMEM;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->graphs.find(graph_id);
    if (it == s->graphs.end() || it->second.retiring || source < 0 ||
        source >= it->second.g->n || (algo == GG_ALGO_SSSP && !it->second.g->weighted)) {
        delete q;
        return GG_EINVAL;
    }
    // the query starts after what the caller enqueued on `stream` so far
    if (!s->spare_events.empty()) {
        q->ready = s->spare_events.back();
        s->spare_events.pop_back();
    } else if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess) {
        delete q;
        return GG_EHIP;
    }
    if (hipEventRecord(q->ready, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        release_event(s, q);
        delete q;
        return GG_EHIP;
    }
    q->id = s->next_query++;
    q->graph_id = graph_id;
    q->algo = algo;
    q->source = source;
    q->out = out_dev;
    q->t_submit = s->now();
    it->second.in_use++;
    s->queue.push_back(q);
    if (query_id) *query_id = q->id;
    s->wake.notify_one();
    return GG_OK;
}

int gg_server_poll(gg_server s, gg_query_result* results, int32_t cap, int32_t* n_done) {
    if (!s || cap < 0 || (cap > 0 && !results)) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int nd = 0;
    while (nd < cap && !s->finished.empty()) {
        results[nd++] = s->finished.front();
        s->finished.pop_front();
    }
    if (n_done) *n_done = nd;
    return GG_OK;
}

int gg_server_state(gg_server s, int32_t* queued, int32_t* in_flight, int64_t* state_bytes) {
    // (results finished but not yet polled are not counted)
    if (!s) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int32_t)s->queue.size();
    if (in_flight) *in_flight = (int32_t)s->active.size();
    if (state_bytes) *state_bytes = s->used;
    return GG_OK;
}

double gg_server_now(gg_server s) { return s ? s->now() : 0.0; }

int gg_server_free(gg_server s) {
    if (!s) return GG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->wake.notify_one();
    if (s->driver.joinable()) s->driver.join();
    (void)hipDeviceSynchronize();
    for (Query* q : s->queue) {
        release_event(s, q);
        delete q;
    }
    for (Query* q : s->active) {
        release_event(s, q);
        delete q;
    }
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    for (auto& kv : s->graphs) free_graph_entry(kv.second);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    delete s;
    return GG_OK;
}

}  // extern "C"
