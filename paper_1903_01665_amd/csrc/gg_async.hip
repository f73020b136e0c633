// gg_async.hip -- host-asynchronous traversal calls (declared in include/gg.h).
//
// The paper's asynchronous execution (Sec. 3.2) removes the host barrier
// between independent kernels, so that one host thread can have BFS and SSSP
// of the same graph in flight together.  A traversal here is a data-
// dependent number of rounds: the host learns that it has ended only from
// the device.  These calls therefore hand the traversal to one driver thread
// of the library and return at once with a ticket.
//
// The rounds run on one of a few streams of the library, taken in turn,
// ordered after everything the caller enqueued on its stream before the call
// (an event recorded there) and after the workspace's previous traversal.
// The driver thread keeps two batches of rounds in flight per traversal and
// reads their completion from pinned host words written by marker kernels
// (no runtime call while it polls), launching the next batch of each
// traversal as soon as the previous one has completed.  The caller's stream
// is never made to wait on work that is not yet enqueued: a stream blocked
// that way could share a hardware queue with the rounds it waits for.

#include <condition_variable>
#include <new>
#include <thread>
#include <vector>

#include "gg_runtime.h"

using namespace gg;

struct gg_ticket_s {
    Drive d;
    gg_graph g = nullptr;
    hipEvent_t ev_in = nullptr;     // on the caller's stream at the call
    hipEvent_t ev_begin = nullptr;  // timing events on the traversal's stream:
    hipEvent_t ev_end = nullptr;    // before the init kernel, after the last round
    int status = GG_OK;
    long long rounds = 0;
    bool done = false;  // guarded by the engine's mutex
};

namespace {

// Streams the traversals run on, taken in turn by the calls.  They are made
// once, with the driver thread: creating a stream can wait for the device,
// which must not happen while traversals of earlier calls run.
constexpr int kAsyncStreams = 8;

struct Engine {
    std::mutex mu;  // guards everything below except the driver's own list
    std::condition_variable work;  // a traversal arrived, or stop
    std::condition_variable done;  // a traversal ended
    std::vector<gg_ticket> pending;  // handed over by callers, not yet taken by the driver
    std::thread th;
    bool stop = false;
    bool started = false;
    int device = 0;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::vector<hipEvent_t> spare_plain, spare_timed;  // events of freed tickets
    ~Engine() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        work.notify_all();
        if (th.joinable()) th.join();
    }
};

Engine& engine() {
    static Engine e;
    return e;
}

// End of a traversal (driver thread, no lock held): the workspace's end
// event and the ticket's timing event go on its stream, the workspace is
// released; the caller sees the ticket done once the driver has marked it
// under the lock.
void finish_traversal(gg_ticket t, int rc) {
    Plan& p = t->d.p;
    gg_ws ws = p.ws;
    int status = rc < 0 ? rc : t->d.status;
    hipError_t e = hipEventRecord(ws->finished, p.s);
    if (e == hipSuccess) e = hipEventRecord(t->ev_end, p.s);
    if (e != hipSuccess && status == GG_OK) status = fail_hip(p.g, e);
    // round stamps of the workspace's next traversal start after this one's
    ws->epoch = std::max(ws->epoch,
                         (int)std::min<long long>(t->d.stamp_base + t->d.r + 1, 1LL << 30));
    record_last(p, status, t->d.r);
    t->status = status;
    t->rounds = t->d.r;
    t->g->n_async.fetch_sub(1);
    ws->busy.store(false);
}

// The driver: sleeps while nothing is in flight; otherwise takes over the
// traversals callers handed in and advances every traversal it holds by at
// most one batch per pass, yielding between passes that change nothing.  The
// lock is held only to take new traversals and to mark ended ones: polling
// and launching happen outside it, so a caller handing in a traversal never
// waits behind the driver's work.
void engine_loop(Engine* E) {
    (void)hipSetDevice(E->device);
    std::vector<gg_ticket> mine, ended;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(E->mu);
            if (mine.empty())
                E->work.wait(lk, [&] { return E->stop || !E->pending.empty(); });
            if (E->stop) return;
            mine.insert(mine.end(), E->pending.begin(), E->pending.end());
            E->pending.clear();
        }
        bool moved = false;
        for (size_t i = 0; i < mine.size();) {
            gg_ticket t = mine[i];
            const long long r0 = t->d.r;
            const int rc = drive_step(t->d, false);
            if (rc == 0) {
                moved |= t->d.r != r0;
                ++i;
                continue;
            }
            finish_traversal(t, rc);
            ended.push_back(t);
            mine[i] = mine.back();
            mine.pop_back();
        }
        if (!ended.empty()) {
            {
                std::lock_guard<std::mutex> lk(E->mu);
                for (gg_ticket t : ended) t->done = true;
            }
            ended.clear();
            E->done.notify_all();
        } else if (!moved) {
            std::this_thread::yield();
        }
    }
}

// Return a ticket's events to the engine for later tickets and delete it.
void free_ticket(gg_ticket t) {
    Engine& E = engine();
    {
        std::lock_guard<std::mutex> lk(E.mu);
        if (t->ev_in) E.spare_plain.push_back(t->ev_in);
        if (t->ev_begin) E.spare_timed.push_back(t->ev_begin);
        if (t->ev_end) E.spare_timed.push_back(t->ev_end);
    }
    delete t;
}

hipError_t take_event(std::vector<hipEvent_t>& spare, bool timed, hipEvent_t* ev) {
    if (!spare.empty()) {
        *ev = spare.back();
        spare.pop_back();
        return hipSuccess;
    }
    return timed ? hipEventCreate(ev) : hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

// Start the driver thread and make the streams (first call); pick a stream
// and the ticket's events.  Engine lock held.
int engine_prepare_locked(Engine& E, gg_ticket t, hipStream_t* s) {
    if (!E.started) {
        E.device = device().id;
        for (int i = 0; i < kAsyncStreams; ++i) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return GG_EHIP;
            E.streams.push_back(st);
        }
        try {
            E.th = std::thread(engine_loop, &E);
        } catch (...) {
            return GG_ENOMEM;
        }
        E.started = true;
    }
    *s = E.streams[E.next_stream];
    E.next_stream = (E.next_stream + 1) % kAsyncStreams;
    hipError_t e = take_event(E.spare_plain, false, &t->ev_in);
    if (e == hipSuccess) e = take_event(E.spare_timed, true, &t->ev_begin);
    if (e == hipSuccess) e = take_event(E.spare_timed, true, &t->ev_end);
    return e == hipSuccess ? GG_OK : GG_EHIP;
}

int run_async(gg_graph g, gg_ws ws, int algo, int source, const gg_opts* opts, int* out,
              void* stream, gg_ticket* ticket) {
    if (!ticket) return GG_EINVAL;
    *ticket = nullptr;
    const hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    Plan p;
    int rc = plan_make(g, ws, algo, source, nullptr, 0, opts, out, nullptr, &p);
    if (rc != GG_OK) return rc;
    ws = p.ws;
    WsClaim claim(ws);
    if (!claim.held()) return GG_EBUSY;
    gg_ticket t = new (std::nothrow) gg_ticket_s();
    if (!t) return GG_ENOMEM;
    t->g = g;
    Engine& E = engine();
    {
        std::lock_guard<std::mutex> lk(E.mu);
        rc = engine_prepare_locked(E, t, &p.s);
    }
    if (rc != GG_OK) {
        free_ticket(t);
        return rc;
    }
    // after the caller's earlier work, and after the workspace's last traversal
    hipError_t e = hipEventRecord(t->ev_in, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(p.s, t->ev_in, 0);
    if (e == hipSuccess && ws->used && ws->last_stream != p.s)
        e = hipStreamWaitEvent(p.s, ws->finished, 0);
    if (e != hipSuccess) {
        free_ticket(t);
        return fail_hip(g, e);
    }
    e = hipEventRecord(t->ev_begin, p.s);
    p.prof = (p.o.flags & GG_OPT_PROFILE) != 0;
    ws->profiled = p.prof;
    ws->nlaunch = 0;
    int base = 0;
    if (e == hipSuccess) base = reserve_stamps(ws, p.s, (long long)g->n + 3, &e);
    if (e == hipSuccess) {
        p.R.epoch = base;
        e = plan_init(p);
    }
    if (e != hipSuccess) {
        (void)hipEventRecord(ws->finished, p.s);
        ws->last_stream = p.s;
        ws->used = true;
        free_ticket(t);
        return fail_hip(g, e);
    }
    t->d.p = p;
    t->d.poll = true;
    rc = drive_start(t->d, 0, base, base);
    if (rc != GG_OK) {
        // the kernels already enqueued are ordered before the next use of
        // the workspace by its end event
        (void)hipEventRecord(ws->finished, p.s);
        ws->last_stream = p.s;
        ws->used = true;
        free_ticket(t);
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(E.mu);
        g->n_async.fetch_add(1);
        claim.keep();
        E.pending.push_back(t);
    }
    E.work.notify_one();
    *ticket = t;
    return GG_OK;
}

// Host wait until the driver has ended the traversal (the end found, or out
// of rounds or time); the device may still run the rounds enqueued past it.
void wait_ended(gg_ticket t) {
    Engine& E = engine();
    std::unique_lock<std::mutex> lk(E.mu);
    E.done.wait(lk, [&] { return t->done; });
}

}  // namespace

extern "C" {

int gg_sssp_async(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts,
                  int32_t* dist_out_dev, void* stream, gg_ticket* ticket) {
    return run_async(g, ws, GG_ALGO_SSSP, source, opts, dist_out_dev, stream, ticket);
}

int gg_bfs_async(gg_graph g, gg_ws ws, int32_t source, const gg_opts* opts, int32_t* dist_out_dev,
                 void* stream, gg_ticket* ticket) {
    return run_async(g, ws, GG_ALGO_BFS, source, opts, dist_out_dev, stream, ticket);
}

int gg_cc_async(gg_graph g, gg_ws ws, const gg_opts* opts, int32_t* label_out_dev, void* stream,
                gg_ticket* ticket) {
    return run_async(g, ws, GG_ALGO_CC, 0, opts, label_out_dev, stream, ticket);
}

int gg_ticket_query(gg_ticket t) {
    if (!t) return GG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(engine().mu);
        if (!t->done) return GG_EBUSY;
    }
    const hipError_t q = hipEventQuery(t->ev_end);
    if (q == hipErrorNotReady) return GG_EBUSY;
    if (q != hipSuccess) return GG_EHIP;
    return t->status;
}

int gg_ticket_wait(gg_ticket t) {
    if (!t) return GG_EINVAL;
    wait_ended(t);
    if (hipEventSynchronize(t->ev_end) != hipSuccess) return GG_EHIP;
    return t->status;
}

int gg_ticket_stream_wait(gg_ticket t, void* stream) {
    if (!t) return GG_EINVAL;
    wait_ended(t);
    if (hipStreamWaitEvent(reinterpret_cast<hipStream_t>(stream), t->ev_end, 0) != hipSuccess)
        return GG_EHIP;
    return t->status;
}

int gg_ticket_times(gg_ticket t, gg_ticket ref, float* begin_ms, float* end_ms, int32_t* rounds) {
    if (!t) return GG_EINVAL;
    if (!ref) ref = t;
    wait_ended(t);
    wait_ended(ref);
    if (hipEventSynchronize(t->ev_end) != hipSuccess ||
        hipEventSynchronize(ref->ev_end) != hipSuccess)
        return GG_EHIP;
    float b = 0.f, e = 0.f;
    if (hipEventElapsedTime(&b, ref->ev_begin, t->ev_begin) != hipSuccess ||
        hipEventElapsedTime(&e, ref->ev_begin, t->ev_end) != hipSuccess)
        return GG_EHIP;
    if (begin_ms) *begin_ms = b;
    if (end_ms) *end_ms = e;
    if (rounds) *rounds = (int32_t)t->rounds;
    return GG_OK;
}

int gg_ticket_free(gg_ticket t) {
    if (!t) return GG_EINVAL;
    wait_ended(t);
    (void)hipEventSynchronize(t->ev_end);  // its failure was reported by the wait calls
    free_ticket(t);
    return GG_OK;
}

}  // extern "C"
