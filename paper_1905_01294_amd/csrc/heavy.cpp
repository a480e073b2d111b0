// Edge-chunk tables of high in-degree vertices for the bottom-up hops.  A hub
// scanned by one wave would serialise thousands of dependent rounds; cut into
// fixed-size chunks it is shared by as many waves as it has chunks.
//
// A table is rebuilt when its threshold option changes.  Callers take a copy
// of the table's description and launch kernels on it later, possibly while
// another thread changes the threshold, so a replaced table is not freed: it
// is retired and released with the graph.  Retired tables are few (one per
// threshold ever used) and small (one record per 256 or 1024 in-edges of the
// vertices above the threshold).
#include <algorithm>
#include <vector>

#include "khop_impl.h"

namespace khop {

static void free_table(HeavyTable &t) {
    if (t.d_vert) (void)hipFree(t.d_vert);
    if (t.d_begin) (void)hipFree(t.d_begin);
    if (t.d_end) (void)hipFree(t.d_end);
    t = HeavyTable{};
}

static HeavyTable build(khop_graph *g, HeavyTable &t, int threshold, int64_t chunk) {
    std::lock_guard<std::mutex> lk(g->heavy_mu);
    if (t.threshold == threshold && t.chunk == chunk) return t;
    HeavyTable nt;
    // Items go chunk-major: the first chunk of every heavy vertex, then the
    // second of every vertex that has one, and so on.  Waves take items in
    // order, so a vertex's later chunks mostly start after its first one has
    // finished, and a chunk whose vertex an earlier chunk already settled
    // (found, or holding every needed bit) stops after one load.
    std::vector<int64_t> at;  // at[j]: first item of the j-th chunks
    int64_t items = 0;
    {
        std::vector<int64_t> nchunks;  // vertices with exactly c chunks, at c
        for (int64_t v = 0; v < g->n; ++v) {
            const int64_t d = g->h_indeg[v];
            if (d <= threshold) continue;
            const int64_t c = (d + chunk - 1) / chunk;
            if ((int64_t)nchunks.size() <= c) nchunks.resize((size_t)c + 1, 0);
            ++nchunks[(size_t)c];
            items += c;
        }
        // the j-th chunks number the vertices with more than j chunks
        at.assign(nchunks.size(), 0);
        int64_t more = 0, pos = items;
        for (size_t c = nchunks.size(); c-- > 1;) {
            more += nchunks[c];
            pos -= more;
            at[c - 1] = pos;
        }
    }
    std::vector<int32_t> vert((size_t)items);
    std::vector<int64_t> begin((size_t)items), end((size_t)items);
    int64_t off = 0;
    for (int64_t v = 0; v < g->n; ++v) {
        const int64_t d = g->h_indeg[v];
        if (d > threshold)
            for (int64_t j = 0; j * chunk < d; ++j) {
                const int64_t i = at[(size_t)j]++;
                vert[(size_t)i] = (int32_t)v;
                begin[(size_t)i] = off + j * chunk;
                end[(size_t)i] = std::min(off + d, off + (j + 1) * chunk);
            }
        off += d;
    }
    nt.threshold = threshold;
    nt.chunk = chunk;
    nt.n = (int64_t)vert.size();
    if (nt.n > 0) {
        if (hipMalloc(&nt.d_vert, vert.size() * 4) != hipSuccess ||
            hipMalloc(&nt.d_begin, begin.size() * 8) != hipSuccess ||
            hipMalloc(&nt.d_end, end.size() * 8) != hipSuccess) {
            (void)hipGetLastError();
            free_table(nt);
            fail(KHOP_ENOMEM, "device allocation for a heavy-vertex chunk table failed");
        }
        try {
            KHOP_HIP(hipMemcpy(nt.d_vert, vert.data(), vert.size() * 4, hipMemcpyHostToDevice));
            KHOP_HIP(hipMemcpy(nt.d_begin, begin.data(), begin.size() * 8, hipMemcpyHostToDevice));
            KHOP_HIP(hipMemcpy(nt.d_end, end.data(), end.size() * 8, hipMemcpyHostToDevice));
        } catch (...) {
            free_table(nt);
            throw;
        }
    }
    // kernels already queued (or about to be, from a copy) may still read the old table
    if (t.threshold >= 0) g->heavy_retired.push_back(t);
    t = nt;
    return t;
}

// 256-edge chunks: one round of 4 in-edges per lane of a wave
HeavyTable plain_heavy_table(khop_graph *g, int threshold) { return build(g, g->plain_heavy, threshold, 256); }

// One table per threshold, kept until the graph is freed: the batched hops
// of one run use several (the threshold grows with the lanes per vertex), and
// each holds one record per 1024 in-edges of its heavy vertices.
HeavyTable batch_heavy_table(khop_graph *g, int threshold) {
    {
        std::lock_guard<std::mutex> lk(g->heavy_mu);
        for (const auto &t : g->batch_heavy)
            if (t.threshold == threshold) return t;
    }
    HeavyTable t;
    build(g, t, threshold, 1024);
    std::lock_guard<std::mutex> lk(g->heavy_mu);
    for (const auto &x : g->batch_heavy)
        if (x.threshold == threshold) {  // built meanwhile by another thread
            g->heavy_retired.push_back(t);
            return x;
        }
    g->batch_heavy.push_back(t);
    return t;
}

HeavyTable plain_heavy_table_current(khop_graph *g) {
    std::lock_guard<std::mutex> lk(g->heavy_mu);
    return g->plain_heavy;
}

// A stable counting sort of the vertices by in-degree: the bottom-up batched
// kernel gives each wave vertices of one degree, so that no lane of a wave
// waits for a longer scan of another.
const int32_t *in_degree_order(khop_graph *g, int64_t *zero) {
    std::lock_guard<std::mutex> lk(g->heavy_mu);
    if (g->d_in_order || g->n == 0) {
        if (zero) *zero = g->in_order_zero;
        return g->d_in_order;
    }
    int64_t maxd = 0;
    for (int64_t v = 0; v < g->n; ++v) maxd = std::max(maxd, g->h_indeg[v]);
    std::vector<int64_t> start((size_t)maxd + 2, 0);
    for (int64_t v = 0; v < g->n; ++v) ++start[(size_t)g->h_indeg[v] + 1];
    for (size_t d = 1; d < start.size(); ++d) start[d] += start[d - 1];
    const int64_t zero_deg = start[1];  // vertices of in-degree 0
    std::vector<int32_t> order((size_t)g->n);
    for (int64_t v = 0; v < g->n; ++v) order[(size_t)start[(size_t)g->h_indeg[v]]++] = (int32_t)v;
    int32_t *d = nullptr;
    if (hipMalloc(&d, order.size() * 4) != hipSuccess) {
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation for the in-degree order failed");
    }
    if (hipMemcpy(d, order.data(), order.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(d);
        fail(KHOP_EINTERNAL, "copy of the in-degree order failed");
    }
    g->d_in_order = d;
    g->in_order_zero = zero_deg;
    if (zero) *zero = g->in_order_zero;
    return d;
}

// Called by graph_free after the device has finished all work.
void heavy_tables_free(khop_graph *g) {
    std::lock_guard<std::mutex> lk(g->heavy_mu);
    if (g->d_in_order) (void)hipFree(g->d_in_order);
    g->d_in_order = nullptr;
    free_table(g->plain_heavy);
    for (auto &t : g->batch_heavy) free_table(t);
    g->batch_heavy.clear();
    for (auto &t : g->heavy_retired) free_table(t);
    g->heavy_retired.clear();
}

Params params_of(khop_graph *g) {
    std::lock_guard<std::mutex> lk(g->params_mu);
    return g->params;
}

void params_set(khop_graph *g, const Params &p) {
    std::lock_guard<std::mutex> lk(g->params_mu);
    g->params = p;
}

}  // namespace khop
