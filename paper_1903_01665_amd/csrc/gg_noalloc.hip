// gg_noalloc.hip -- BFS without any allocation in the call (gg_bfs_noalloc
// in include/gg.h), for callers that cannot allocate device memory.
//
// The traversal's scratch memory -- frontier flags, heavy-row bits, the
// control block, per-block counters and push counts, the end word, and the
// levels in the library's vertex order when the graph is renumbered -- lives
// in one file-scope device array of fixed size instead of a workspace.  Each
// device holds its own copy of the array; its address on a device is taken
// once, with that device current, at the first call there, and only that
// address is used from the host afterwards.  Calls are serialised per
// device by a lock, and each call returns only after every kernel it
// enqueued has completed, so no call ever sees another one's kernels; the
// array keeps the last call's contents.

#include <mutex>

#include "gg_runtime.h"

using namespace gg;

namespace {

constexpr long long kNaMaxN = 1LL << 22;  // vertices at most
constexpr long long kNaTiles = (kNaMaxN + 63) / 64;
constexpr long long kNaVBytes = ((kNaTiles + 63) / 64) * 64 * 64;  // vertex flags, one generation
constexpr long long kNaTBytes = ((kNaTiles + 63) / 64) * 64;       // tile flags, one generation

constexpr long long align256(long long x) { return (x + 255) & ~255LL; }

// byte offsets of the parts of the array
constexpr long long kOffVflag = 0;
constexpr long long kOffTflag = 2 * kNaVBytes;
constexpr long long kNaHWords = (kNaMaxN + 31) / 32;  // heavy-row bits, one generation
constexpr long long kOffHbits = align256(kOffTflag + 2 * kNaTBytes);
constexpr long long kOffCtl = align256(kOffHbits + 4 * 2 * kNaHWords);
constexpr long long kOffStat = align256(kOffCtl + (long long)sizeof(Ctl));
constexpr long long kOffCount = align256(kOffStat + (long long)sizeof(Stat) * kKinds * kMaxStatBlocks);
constexpr long long kOffDone = align256(kOffCount + 4LL * 3 * 2 * kMaxStatBlocks);
constexpr long long kOffRval = align256(kOffDone + 16);  // levels of a renumbered graph
constexpr long long kNaBytes = align256(kOffRval + 4 * kNaMaxN);

}  // namespace

// about 27 MB on every device the library runs on, held until the process ends
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

__global__ __launch_bounds__(256) void k_fill_words(int* p, long long count, int value) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long i = tid; i < count; i += tt) p[i] = value;
}

constexpr int kMaxDevices = 64;

struct NaDevice {
    bool ready = false;
    unsigned char* ptr = nullptr;  // the device address of `scratch` on this device
    int epoch = 0;                 // tag of the next call
};

std::mutex g_na_mu;
NaDevice g_na[kMaxDevices];

// Address of this device's copy of the array, the first time a call runs on
// the device.
int na_setup(int dev) {
    NaDevice& d = g_na[dev];
    if (d.ready) return GG_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GG_EHIP;
    d.ptr = static_cast<unsigned char*>(p);
    d.epoch = 0;
    d.ready = true;
    return GG_OK;
}

}  // namespace

extern "C" int gg_bfs_noalloc(gg_graph g, int32_t source, const gg_opts* opts,
                              int32_t* dist_out_dev, void* stream) {
    if (!g) return GG_EINVAL;
    if ((long long)g->n > kNaMaxN) return GG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GG_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return GG_ENOTSUP;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_na_mu);
    int rc = na_setup(dev);
    if (rc != GG_OK) return rc;
    NaDevice& D = g_na[dev];

    // a workspace view of the array (the host side of it lives on the stack)
    gg_ws_s w;
    w.owner = g;
    w.dev.vflag[0] = D.ptr + kOffVflag;
    w.dev.vflag[1] = D.ptr + kOffVflag + kNaVBytes;
    w.dev.tflag[0] = D.ptr + kOffTflag;
    w.dev.tflag[1] = D.ptr + kOffTflag + kNaTBytes;
    w.dev.hbits[0] = reinterpret_cast<unsigned*>(D.ptr + kOffHbits);
    w.dev.hbits[1] = w.dev.hbits[0] + kNaHWords;
    w.dev.ctl = reinterpret_cast<Ctl*>(D.ptr + kOffCtl);
    w.dev.stat = reinterpret_cast<Stat*>(D.ptr + kOffStat);
    w.dev.pcount = reinterpret_cast<int*>(D.ptr + kOffCount);
    w.rval = g->renumbered ? reinterpret_cast<int*>(D.ptr + kOffRval) : nullptr;
    int* done_word = reinterpret_cast<int*>(D.ptr + kOffDone);

    Plan p;
    rc = plan_make(g, &w, GG_ALGO_BFS, source, nullptr, 0, opts, dist_out_dev, s, &p);
    if (rc != GG_OK) return rc;
    p.prof = false;  // profiling would create events
    // the end word is in the array: read back with a copy, not polled
    p.R.host_done = done_word;

    // the call's tag (tags restart long before the int range ends)
    const long long span = (long long)g->n + 3;
    if ((long long)D.epoch + span > (1LL << 30)) D.epoch = 0;
    const int base = D.epoch;
    p.R.epoch = base;
    // the end word holds the last call's tag: reset it before any round runs
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(64), 0, s, done_word, 1LL, -1);
    HIPCHK(g, hipGetLastError());
    HIPCHK(g, plan_init(p));

    // batches of rounds doubling up to kMaxBatch; after each, the end word is
    // copied back and the stream drained, so nothing of this call is left on
    // the stream when it returns
    const long long limit = max_rounds(p);
    const auto t0 = std::chrono::steady_clock::now();
    long long r = 0;
    int batch = 2, status = GG_OK, seen = -1;
    for (;;) {
        const long long stop = std::min(r + batch, limit);
        for (; r < stop; ++r) HIPCHK(g, plan_round(p, (int)r));
        HIPCHK(g, hipMemcpyAsync(&seen, done_word, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(g, hipStreamSynchronize(s));
        if (seen == base) break;
        const long long ms = std::chrono::duration_cast<std::chrono::milliseconds>(
                                 std::chrono::steady_clock::now() - t0).count();
        if (r >= limit) {
            status = GG_EITER;
            break;
        }
        if (ms > p.o.time_limit_ms) {
            status = GG_ETIMEOUT;
            break;
        }
        batch = std::min(batch * 2, kMaxBatch);
    }
    D.epoch = (int)std::min<long long>((long long)base + r + 1, 1LL << 30);
    // a renumbered graph: the levels to the caller's order
    if (p.renum) {
        HIPCHK(g, plan_finish(p));
        HIPCHK(g, hipStreamSynchronize(s));
    }
    return status;
}
