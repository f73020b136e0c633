// gg_sort.hip -- upload helper: the edges of every row ordered by head.
//
// On a renumbered (hottest-first) graph the heads of a long row spread over
// the whole id range in the caller's edge order, so the 64 head values a
// wavefront gathers at once fall in about 61 different 128-byte lines on
// rmat22's rows longer than 16 edges.  With each row's edges ordered by
// head the same gathers touch about 33 lines: the hot heads (small ids)
// come first and share lines, and the rest are at least in increasing
// order.  The order of edges within a row changes no traversal result; the
// forest keeps its keys through the edge maps, which follow the edges.
// The sort is rocPRIM's segmented radix sort (one segment per row, keys =
// heads, values = the edges' places), used here at upload only.

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "gg_runtime.h"

namespace gg {

namespace {

__global__ __launch_bounds__(256) void k_iota(int* p, int m) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long e = tid; e < m; e += tt) p[e] = (int)e;
}

// Edge p of the sorted order came from place perm[p]: move its weight and
// caller index along, and point the caller edge back at its new place.
__global__ __launch_bounds__(256) void k_apply_order(const int* perm, int m, const int* w_in,
                                                     int* w_out, const int* eorig_in,
                                                     int* eorig_out, int* epos) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tt = (long long)gridDim.x * blockDim.x;
    for (long long p = tid; p < m; p += tt) {
        const int q = perm[p];
        if (w_in) w_out[p] = w_in[q];
        if (eorig_in) {
            const int eo = eorig_in[q];
            eorig_out[p] = eo;
            epos[eo] = (int)p;
        }
    }
}

}  // namespace

int sort_rows_by_head(gg_graph g, hipStream_t s) {
    const int n = g->n;
    const long long m = g->m;
    if (m < 2) return GG_OK;
    int bits = 1;
    while (bits < 31 && (1LL << bits) < n) ++bits;
    int *kout = nullptr, *vin = nullptr, *vout = nullptr, *wout = nullptr, *eout = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    auto done = [&](hipError_t e) {
        (void)hipStreamSynchronize(s);
        dfree(kout);
        dfree(vin);
        dfree(vout);
        dfree(wout);
        dfree(eout);
        if (tmp) (void)hipFree(tmp);
        return e == hipSuccess ? GG_OK : e == hipErrorOutOfMemory ? GG_ENOMEM : GG_EHIP;
    };
    hipError_t e = rocprim::segmented_radix_sort_pairs(
        nullptr, tmp_bytes, g->col, (int*)nullptr, (int*)nullptr, (int*)nullptr, (unsigned)m,
        (unsigned)n, g->row, g->row + 1, 0, (unsigned)bits, s);
    if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 1));
    if (e == hipSuccess) e = dalloc(&kout, (size_t)m);
    if (e == hipSuccess) e = dalloc(&vin, (size_t)m);
    if (e == hipSuccess) e = dalloc(&vout, (size_t)m);
    if (e == hipSuccess && g->w) e = dalloc(&wout, (size_t)m);
    if (e == hipSuccess && g->eorig) e = dalloc(&eout, (size_t)m);
    if (e != hipSuccess) return done(e);
    const int grid = (int)std::max(1LL, std::min<long long>((m + 255) / 256, device().max_blocks));
    hipLaunchKernelGGL(k_iota, dim3(grid), dim3(256), 0, s, vin, (int)m);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = rocprim::segmented_radix_sort_pairs(tmp, tmp_bytes, g->col, kout, vin, vout,
                                                (unsigned)m, (unsigned)n, g->row, g->row + 1, 0,
                                                (unsigned)bits, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_apply_order, dim3(grid), dim3(256), 0, s, vout, (int)m, g->w, wout,
                           g->eorig, eout, g->epos);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(e);
    std::swap(g->col, kout);
    if (g->w) std::swap(g->w, wout);
    if (g->eorig) std::swap(g->eorig, eout);
    return done(hipSuccess);  // frees the old arrays (now in kout, wout, eout)
}

}  // namespace gg
