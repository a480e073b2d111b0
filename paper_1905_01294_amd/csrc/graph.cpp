// Host-side construction of the compressed sparse adjacency matrix (CSR with
// int64 row pointers, int32 column indices, neighbors ascending) from raw edge
// tuples: the graph storage model of the paper's Section II.  Self-loops and
// duplicate tuples carry no adjacency and are dropped.
//
// Parallel bucket sort with std::thread:
//   1. every thread counts its share of arcs per tail-vertex bucket;
//   2. arcs are scattered, bucket by bucket, as packed (tail, head) pairs;
//   3. each bucket is sorted by (tail, head) independently, duplicates removed;
//   4. row pointers come from a prefix over the per-vertex degrees, and each
//      bucket copies its heads into the final column array.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "khop_impl.h"

namespace khop {

int host_threads() {
    if (const char *e = std::getenv("KHOP_THREADS")) {
        int t = std::atoi(e);
        if (t > 0) return t;
    }
    unsigned hc = std::thread::hardware_concurrency();
    int t = hc ? (int)hc : 4;
    return std::min(t, 16);
}

template <class F>
static void parallel_for(int64_t n, int threads, F &&f) {
    if (n <= 0) return;
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
    std::vector<std::thread> pool;
    pool.reserve(threads);
    for (int t = 0; t < threads; ++t) {
        int64_t b = n * t / threads, e = n * (t + 1) / threads;
        pool.emplace_back([&f, t, b, e] { f(t, b, e); });
    }
    for (auto &th : pool) th.join();
}

// Dynamic scheduling over `n` items.
template <class F>
static void parallel_items(int64_t n, int threads, F &&f) {
    std::atomic<int64_t> next{0};
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto &th : pool) th.join();
}

HostCSR build_csr(const int32_t *a, const int32_t *b, int64_t m, int64_t n, bool both) {
    const int T = host_threads();
    // vertex buckets of equal width (a power of two); at least 8 buckets per thread
    int shift = 0;
    while (((n - 1) >> shift) + 1 > (int64_t)T * 8 && shift < 31) ++shift;
    const int64_t nb = ((n - 1) >> shift) + 1;
    // 1. per-thread bucket counts
    std::vector<int64_t> cnt((size_t)T * (size_t)nb, 0);
    parallel_for(m, T, [&](int t, int64_t lo, int64_t hi) {
        int64_t *c = &cnt[(size_t)t * (size_t)nb];
        for (int64_t i = lo; i < hi; ++i) {
            int32_t u = a[i], v = b[i];
            if (u == v) continue;
            c[u >> shift]++;
            if (both) c[v >> shift]++;
        }
    });
    // bucket-major offsets: bucket k, thread t
    std::vector<int64_t> bstart(nb + 1, 0);
    std::vector<int64_t> pos((size_t)T * (size_t)nb);
    {
        int64_t run = 0;
        for (int64_t k = 0; k < nb; ++k) {
            bstart[k] = run;
            for (int t = 0; t < T; ++t) {
                pos[(size_t)t * nb + k] = run;
                run += cnt[(size_t)t * nb + k];
            }
        }
        bstart[nb] = run;
    }
    const int64_t arcs = bstart[nb];
    std::vector<uint64_t> buf((size_t)std::max<int64_t>(arcs, 1));
    // 2. scatter packed (tail << 32 | head); the same split of [0, m) as the count pass
    parallel_for(m, T, [&](int t, int64_t lo, int64_t hi) {
        int64_t *p = &pos[(size_t)t * (size_t)nb];
        for (int64_t i = lo; i < hi; ++i) {
            uint32_t u = (uint32_t)a[i], v = (uint32_t)b[i];
            if (u == v) continue;
            buf[p[u >> shift]++] = ((uint64_t)u << 32) | v;
            if (both) buf[p[v >> shift]++] = ((uint64_t)v << 32) | u;
        }
    });
    // 3. sort + dedup each bucket; per-vertex degrees
    HostCSR out;
    out.n = n;
    out.rowptr.assign((size_t)n + 1, 0);
    std::vector<int64_t> bkeep(nb, 0);
    parallel_items(nb, T, [&](int64_t k) {
        uint64_t *lo = buf.data() + bstart[k], *hi = buf.data() + bstart[k + 1];
        std::sort(lo, hi);
        uint64_t *w = std::unique(lo, hi);
        bkeep[k] = w - lo;
        for (uint64_t *p = lo; p < w; ++p) out.rowptr[(*p >> 32) + 1]++;
    });
    for (int64_t v = 0; v < n; ++v) out.rowptr[v + 1] += out.rowptr[v];
    out.colidx.resize((size_t)out.rowptr[n]);
    // 4. copy heads; bucket k's rows start at rowptr[k << shift]
    parallel_items(nb, T, [&](int64_t k) {
        const uint64_t *lo = buf.data() + bstart[k];
        int64_t dst = out.rowptr[std::min<int64_t>(k << shift, n)];
        for (int64_t i = 0; i < bkeep[k]; ++i) out.colidx[dst + i] = (int32_t)(lo[i] & 0xffffffffu);
    });
    return out;
}

uint64_t csr_hash(const HostCSR &c) {
    // FNV-1a over the sizes and a strided sample plus the full row pointers' last value
    uint64_t h = 1469598103934665603ULL;
    auto mixin = [&](uint64_t x) {
        for (int i = 0; i < 8; ++i) {
            h ^= (x >> (8 * i)) & 0xff;
            h *= 1099511628211ULL;
        }
    };
    mixin((uint64_t)c.n);
    mixin((uint64_t)c.colidx.size());
    const size_t step = std::max<size_t>(1, c.colidx.size() / 65536);
    for (size_t i = 0; i < c.colidx.size(); i += step) mixin((uint64_t)(uint32_t)c.colidx[i]);
    const size_t rstep = std::max<size_t>(1, c.rowptr.size() / 65536);
    for (size_t i = 0; i < c.rowptr.size(); i += rstep) mixin((uint64_t)c.rowptr[i]);
    return h;
}

}  // namespace khop
