// gg_runtime.h -- host-side internals shared by the runtime sources of libgg
// (gg_api.hip, gg_batch.hip): handle structures, device facts, the traversal
// plan and its enqueue functions.  Not part of the public ABI.
#pragma once

#include <gg.h>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <vector>

#include "gg_internal.h"

namespace gg {

constexpr int kVersion = 1;
constexpr int kBlock = 256;
constexpr int kMaxBatch = 16;
constexpr int kDefaultTimeLimitMs = 60000;

struct Dev {
    int id = 0;
    int cus = 0;
    int max_blocks = 0;  // resident blocks of kBlock threads on the whole device
};

inline Dev& device() {
    static Dev d;
    static std::once_flag once;
    std::call_once(once, [] {
        if (hipGetDevice(&d.id) != hipSuccess) d.id = 0;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d.id) == hipSuccess) {
            d.cus = p.multiProcessorCount;
            const int per_cu = std::max(1, p.maxThreadsPerMultiProcessor / kBlock);
            d.max_blocks = std::min(kMaxStatBlocks, d.cus * per_cu);
        }
        if (d.max_blocks <= 0) d.max_blocks = 1024;
    });
    return d;
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace gg

struct gg_ws_s {
    gg_graph owner = nullptr;
    std::atomic<bool> busy{false};  // a host call is using the workspace
    gg::DevWs dev{};
    unsigned char* vflag_mem = nullptr;
    int epoch = 0;  // round stamps of the next traversal start here
    // pinned host words: [0] the tag written by the kernel that finds the
    // end; [2..3] (64 bits) the sequence number of the last batch of rounds
    // completed, written by a marker kernel (non-blocking driving)
    int* h_done = nullptr;
    unsigned long long prog_seq = 0;  // last sequence number enqueued
    // minimum spanning forest: union-find parents and per-root offers,
    // allocated by the first gg_msf call on the workspace
    int* msf_parent = nullptr;
    unsigned long long* msf_best = nullptr;
    // renumbered graph: the traversal's values in the library's vertex order
    // and the per-component minimum of the caller's ids (CC)
    int* rval = nullptr;
    int* rmin = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t finished = nullptr;
    hipStream_t last_stream = nullptr;
    bool used = false;
    gg_stats last{};
    bool is_default = false;
    // GG_OPT_PROFILE: an event pair and a kind per launch of the last call
    std::vector<hipEvent_t> pev;
    std::vector<int> pkind;
    int nlaunch = 0;
    bool profiled = false;
    int rounds = 0;
};

// The 64-bit batch sequence word inside a workspace's pinned block.
inline unsigned long long* prog_word(gg_ws ws) {
    return reinterpret_cast<unsigned long long*>(ws->h_done + 2);
}

struct gg_graph_s {
    int n = 0;
    long long m = 0;
    int max_deg = 0;
    int argmax_deg = 0;  // a vertex of largest out-degree (caller's id)
    int levels = -1;  // BFS rounds from argmax_deg, measured by gg_graph_probe
    bool weighted = false;
    bool has_sym = false;
    bool symmetric = false;
    int err = GG_OK;
    int n_ws = 0;  // user workspaces alive
    std::atomic<int> n_async{0};  // host-asynchronous traversals in flight
    // device arrays
    int *row = nullptr, *col = nullptr, *w = nullptr, *src = nullptr;
    int *srow = nullptr, *scol = nullptr, *ssrc = nullptr;
    int2 *hchunks = nullptr, *shchunks = nullptr;
    int n_hchunks = 0, n_shchunks = 0;
    long long ms = 0;
    int heavy = gg::kHeavyUniform, chunk = gg::kChunk;
    int *psrc = nullptr, *pcol = nullptr, *pw = nullptr;  // head-partitioned edge list
    int *trow = nullptr, *tcol = nullptr, *tw = nullptr;  // weighted in-edge CSR
    int2* tchunks = nullptr;
    int n_tchunks = 0;
    int poff[gg::kXcd + 1] = {};
    // renumbered vertex order (GG_RENUMBER): new id of each caller id and
    // back, on the device, and the new ids on the host (to map sources);
    // the caller's index of each stored edge and the stored place of each
    // caller edge (the forest's keys and output)
    bool renumbered = false;
    int n_active = 0;  // renumbered: vertices with an edge (new ids below this)
    int *newid = nullptr, *oldid = nullptr;
    int *eorig = nullptr, *epos = nullptr;
    std::vector<int> h_newid;
    double avg_w = 0;  // mean edge weight (0 when unweighted)
    int max_w = 0;     // largest edge weight
    gg_ws_s* ws0 = nullptr;
};

namespace gg {

// Holds a workspace for one host call; a second concurrent call on the same
// workspace finds it taken (GG_EBUSY).
struct WsClaim {
    gg_ws_s* ws = nullptr;
    explicit WsClaim(gg_ws_s* w) {
        bool f = false;
        if (w && w->busy.compare_exchange_strong(f, true)) ws = w;
    }
    ~WsClaim() {
        if (ws) ws->busy.store(false);
    }
    bool held() const { return ws != nullptr; }
    // the claim outlives the call (a host-asynchronous traversal releases it
    // when it ends)
    void keep() { ws = nullptr; }
};

inline int fail_hip(gg_graph g, hipError_t e) {
    if (e == hipSuccess) return GG_OK;
    if (g && g->err == GG_OK) g->err = (e == hipErrorOutOfMemory) ? GG_ENOMEM : GG_EHIP;
    return (e == hipErrorOutOfMemory) ? GG_ENOMEM : GG_EHIP;
}

#define HIPCHK(g, call)                                      \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return fail_hip((g), e_);      \
    } while (0)

// A traversal prepared for enqueueing: variant, launch shapes and the round
// template.  The eager driver and graph capture share it.
struct Plan {
    gg_graph g = nullptr;
    gg_ws ws = nullptr;
    int algo = 0;
    gg_opts o{};
    hipStream_t s = nullptr;
    Round R{};
    bool async = false, edge = false, cc = false, diropt = false, uf = false;
    bool need_heavy = false, need_jump = false, prof = false;
    // renumbered graph: R.val is the workspace's array; the finishing
    // kernels write `out` in the caller's order
    bool renum = false;
    int* out = nullptr;
    int src_caller = -1;  // the source as the caller numbers it (-1: CC)
    int g_init = 1, g_seed = 1, g_round = 1, g_heavy = 1, g_jump = 1;
};

// Validate a call and fill the plan (variant resolved, grids sized).
int plan_make(gg_graph g, gg_ws ws, int algo, int source, const int* sources_dev, int nsrc,
              const gg_opts* opts, int* out, hipStream_t s, Plan* P);
// Enqueue the init kernel (and the seed kernel of a multi-source plan).
hipError_t plan_init(Plan& p);
// Enqueue round r (round kernel, heavy-chunk or shortcut kernel as needed).
hipError_t plan_round(Plan& p, int r);
// Enqueue what ends a traversal once its rounds are done: on a renumbered
// graph, the kernels that write the output in the caller's order.
hipError_t plan_finish(Plan& p);
// Reserve `span` round stamps on a workspace; returns the first.
int reserve_stamps(gg_ws ws, hipStream_t s, long long span, hipError_t* err);
// Resumable eager driver of one traversal (see gg_api.hip).
struct Drive {
    Plan p;
    long long r = 0, max_rounds = 0;
    int batch = 2, k = 0;
    // poll: batches end with a marker kernel that stores their sequence
    // number into pinned memory (read without any runtime call); otherwise
    // with an event the host waits on
    bool poll = false;
    unsigned long long seq[2] = {0, 0};
    int stamp_base = 0, tag = 0;
    std::chrono::steady_clock::time_point t0;
    int status = GG_OK;
    bool finished = false;
    // poll: out of rounds or time, waiting for the newer batch to complete
    // before stop_status becomes final
    bool stopping = false;
    int stop_status = GG_OK;
    // poll, renumbered graph: the finishing kernels are enqueued and the
    // traversal ends when the marker after them has run
    bool finishing = false;
    unsigned long long fin_seq = 0;
};
// Bound on the rounds of a traversal planned by p.
long long max_rounds(const Plan& p);
// Enqueue the first two batches of rounds from round r0.
int drive_start(Drive& d, long long r0, int stamp_base, int tag);
// Enqueue the next batch.
int drive_enqueue(Drive& d);
// Advance: 1 = finished (d.status holds GG_OK, GG_EITER or GG_ETIMEOUT),
// 0 = still running (non-blocking form only), < 0 = HIP failure.
int drive_step(Drive& d, bool block);
// Blocking form: rounds from r0 until the end is reported.
int plan_drive(Plan& p, long long r0, int stamp_base, int tag, long long* r_end);
// Upload of a renumbered graph: order each row's edges by head (gg_sort.hip).
int sort_rows_by_head(gg_graph g, hipStream_t s);
// Record the variant, status and round count of a finished call.
void record_last(Plan& p, int status, long long rounds);
// One traversal from one source or from a device list of sources.
int run_multi(gg_graph g, gg_ws ws, int algo, int source, const int* sources_dev, int nsrc,
              const gg_opts* opts, int* out, void* stream);

}  // namespace gg
