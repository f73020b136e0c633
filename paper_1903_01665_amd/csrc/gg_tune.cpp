// gg_tune.cpp -- graph classes and the process-wide tuning table behind the
// AUTO variant choice (declared in include/gg.h).  Host code only.

#include <gg.h>

#include <cmath>
#include <cstdlib>
#include <mutex>
#include <vector>

namespace {

std::mutex g_mu;
std::vector<gg_tune_entry> g_table;

bool valid(const gg_tune_entry& e) {
    return e.algo >= 0 && e.algo <= 2 && e.size_class >= 0 && e.size_class < 64 &&
           e.skew_class >= 0 && e.skew_class <= 2 && e.depth_class >= -1 && e.depth_class <= 2 &&
           (e.mode == GG_VERTEX || e.mode == GG_EDGE) &&
           (e.sched == GG_SYNC || e.sched == GG_ASYNC ||
            (e.sched == GG_NEARFAR && e.algo == GG_ALGO_SSSP && e.mode == GG_VERTEX) ||
            (e.sched == GG_DIROPT && e.algo == GG_ALGO_BFS && e.mode == GG_VERTEX) ||
            (e.sched == GG_DIROPT && e.algo == GG_ALGO_SSSP && e.mode == GG_VERTEX) ||
            (e.sched == GG_DIROPT && e.algo == GG_ALGO_CC) ||
            (e.sched == GG_UNIONFIND && e.algo == GG_ALGO_CC && e.mode == GG_VERTEX)) &&
           e.mapping >= GG_MAP_AUTO && e.mapping <= GG_MAP_BALANCED && e.delta_eighths >= 0 &&
           e.delta_eighths <= 1 << 23 && e.hops >= 0 && e.hops <= 64 && e.far_degree >= 0 &&
           (e.far_degree == 0 || e.sched == GG_NEARFAR) &&
           (e.hops == 0 || (e.mode == GG_VERTEX && (e.sched == GG_ASYNC || e.sched == GG_NEARFAR) &&
                            (e.mapping == GG_MAP_AUTO || e.mapping == GG_MAP_BALANCED)));
}

// Built-in choice, from the measured behaviour of the variants on the
// synthetic workloads (uniform, R-MAT, grid): asynchronous vertex-based
// rounds for SSSP everywhere; BFS synchronous on shallow graphs and
// asynchronous on deep ones; CC by edge sweeps with the shortcut.
void builtin(int algo, int depth, gg_tune_entry* e) {
    e->mapping = GG_MAP_BALANCED;
    e->delta_eighths = 0;
    e->hops = 0;
    e->far_degree = 0;
    if (algo == GG_ALGO_SSSP) {
        e->mode = GG_VERTEX;
        e->sched = GG_ASYNC;
    } else if (algo == GG_ALGO_BFS) {
        e->mode = GG_VERTEX;
        e->sched = depth >= 1 || depth < 0 ? GG_ASYNC : GG_SYNC;
    } else {
        e->mode = GG_EDGE;
        e->sched = GG_SYNC;
    }
}

}  // namespace

extern "C" {

int gg_class_of(int64_t m, int32_t n, int32_t max_out_degree, int32_t levels,
                int32_t* size_class, int32_t* skew_class, int32_t* depth_class) {
    if (n < 1 || m < 0 || max_out_degree < 0 || !size_class || !skew_class || !depth_class)
        return GG_EINVAL;
    int lg = 0;
    for (int64_t x = m > 1 ? m : 1; x > 1; x >>= 1) ++lg;
    *size_class = lg / 2;
    const double avg = (double)m / (double)n;
    const double skew = avg > 0 ? (double)max_out_degree / avg : 0.0;
    *skew_class = skew < 8.0 ? 0 : skew < 128.0 ? 1 : 2;
    *depth_class = levels < 0 ? -1 : levels < 16 ? 0 : levels < 256 ? 1 : 2;
    return GG_OK;
}

int gg_tune_set(const gg_tune_entry* entries, int32_t count) {
    if (count < 0 || (count > 0 && !entries)) return GG_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!valid(entries[i])) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.assign(entries, entries + count);
    return GG_OK;
}

int gg_tune_get(gg_tune_entry* out, int32_t cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int n = (int)g_table.size();
    for (int i = 0; i < n && i < cap && out; ++i) out[i] = g_table[i];
    return n;
}

int gg_tune_lookup(int32_t algo, int32_t size_class, int32_t skew_class, int32_t depth_class,
                   gg_tune_entry* out) {
    if (algo < 0 || algo > 2 || !out) return GG_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1, best_score = 1 << 30;
    for (int i = 0; i < (int)g_table.size(); ++i) {
        const gg_tune_entry& e = g_table[i];
        if (e.algo != algo) continue;
        int score = std::abs(e.size_class - size_class);
        if (e.skew_class != skew_class) score += 4;
        if (e.depth_class >= 0 && depth_class >= 0 && e.depth_class != depth_class) score += 4;
        if (score < best_score) {
            best_score = score;
            best = i;
        }
    }
    gg_tune_entry r{};
    if (best < 0) {
        builtin(algo, depth_class, &r);
    } else {
        r = g_table[best];
        if (r.mapping == GG_MAP_AUTO) r.mapping = GG_MAP_BALANCED;
    }
    r.algo = algo;
    r.size_class = size_class;
    r.skew_class = skew_class;
    r.depth_class = depth_class;
    *out = r;
    return GG_OK;
}

}  // extern "C"
