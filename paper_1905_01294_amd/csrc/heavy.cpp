// Edge-chunk tables of high in-degree vertices for the bottom-up hops.  A hub
// scanned by one wave would serialise thousands of dependent rounds; cut into
// fixed-size chunks it is shared by as many waves as it has chunks.
#include <algorithm>

#include "khop_impl.h"

namespace khop {

static void free_table(HeavyTable &t) {
    if (t.d_vert) (void)hipFree(t.d_vert);
    if (t.d_begin) (void)hipFree(t.d_begin);
    if (t.d_end) (void)hipFree(t.d_end);
    t = HeavyTable{};
}

static const HeavyTable &build(khop_graph *g, HeavyTable &t, int threshold, int64_t chunk) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (t.threshold == threshold && t.chunk == chunk) return t;
    // the previous table may still be read by queued kernels
    KHOP_HIP(hipDeviceSynchronize());
    free_table(t);
    std::vector<int32_t> vert;
    std::vector<int64_t> begin, end;
    {
        int64_t items = 0;
        for (int64_t v = 0; v < g->n; ++v)
            if (g->h_indeg[v] > threshold) items += (g->h_indeg[v] + chunk - 1) / chunk;
        vert.reserve((size_t)items);
        begin.reserve((size_t)items);
        end.reserve((size_t)items);
    }
    int64_t off = 0;
    for (int64_t v = 0; v < g->n; ++v) {
        const int64_t d = g->h_indeg[v];
        if (d > threshold)
            for (int64_t b = off; b < off + d; b += chunk) {
                vert.push_back((int32_t)v);
                begin.push_back(b);
                end.push_back(std::min(off + d, b + chunk));
            }
        off += d;
    }
    t.threshold = threshold;
    t.chunk = chunk;
    t.n = (int64_t)vert.size();
    if (t.n > 0) {
        if (hipMalloc(&t.d_vert, vert.size() * 4) != hipSuccess || hipMalloc(&t.d_begin, begin.size() * 8) != hipSuccess ||
            hipMalloc(&t.d_end, end.size() * 8) != hipSuccess) {
            (void)hipGetLastError();
            free_table(t);
            fail(KHOP_ENOMEM, "device allocation for a heavy-vertex chunk table failed");
        }
        KHOP_HIP(hipMemcpy(t.d_vert, vert.data(), vert.size() * 4, hipMemcpyHostToDevice));
        KHOP_HIP(hipMemcpy(t.d_begin, begin.data(), begin.size() * 8, hipMemcpyHostToDevice));
        KHOP_HIP(hipMemcpy(t.d_end, end.data(), end.size() * 8, hipMemcpyHostToDevice));
    }
    return t;
}

// 256-edge chunks: one round of 4 in-edges per lane of a wave
const HeavyTable &plain_heavy_table(khop_graph *g) { return build(g, g->plain_heavy, g->params.pull_heavy, 256); }

const HeavyTable &batch_heavy_table(khop_graph *g) { return build(g, g->batch_heavy, g->params.batch_heavy, 1024); }

void heavy_tables_free(khop_graph *g) {
    free_table(g->plain_heavy);
    free_table(g->batch_heavy);
}

}  // namespace khop
