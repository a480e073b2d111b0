// The library's C ABI (declared in include/khop.h): argument validation,
// error mapping, graph lifetime, pooled query contexts and profiling.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>

#include "khop_impl.h"
#include "serve_policy.h"

namespace khop {

static thread_local std::string t_err;

void fail(int status, const std::string &msg) { throw Error{status, msg}; }

void set_last_error(const std::string &msg) { t_err = msg; }

void hip_fail(hipError_t e, const char *what, const char *file, int line) {
    const char *base = std::strrchr(file, '/');
    std::string m = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what +
                    " at " + (base ? base + 1 : file) + ":" + std::to_string(line);
    throw Error{e == hipErrorOutOfMemory ? KHOP_ENOMEM : KHOP_EDEVICE, m};
}

const char *const kKernelNames[KK_COUNT_KINDS] = {
    "plain_init", "plain_step", "plain_hop_push", "plain_hop_pull", "plain_compact", "batch_init", "batch_push",
    "batch_pull", "batch_pull_heavy", "batch_count", "plain_set", "plain_degree", "empty_launch"};

template <class F>
static int guard(F &&f) {
    try {
        f();
        return KHOP_OK;
    } catch (const Error &e) {
        t_err = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        t_err = "host allocation failed";
        return KHOP_ENOMEM;
    } catch (const std::exception &e) {
        t_err = std::string("internal error: ") + e.what();
        return KHOP_EINTERNAL;
    } catch (...) {
        t_err = "internal error";
        return KHOP_EINTERNAL;
    }
}

// Picks the first gfx950 device; fails with KHOP_EDEVICE when there is none.
static int require_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        fail(KHOP_EDEVICE, "no HIP device available");
    }
    for (int d = 0; d < count; ++d) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) != hipSuccess) continue;
        if (std::strncmp(p.gcnArchName, "gfx950", 6) == 0) return d;
    }
    fail(KHOP_EDEVICE, "no gfx950 device found");
}

static void check_graph(const khop_graph *g) {
    if (!g) fail(KHOP_EINVAL, "graph is NULL");
}

// ---------------------------------------------------------------- profiling

ProfScope::ProfScope(khop_graph *g, int kind, hipStream_t st) : g_(g), kind_(kind), st_(st) {
    if (!g) return;  // an unprofiled launch
    Profiler &P = g->prof;
    if (!P.on) return;
    std::lock_guard<std::mutex> lk(g->prof_mu);
    if (!P.on) return;
    if (P.next_slot >= P.cap) prof_collect(g);
    slot_ = P.next_slot++;
    units_ = P.d_units + 4 * 64 * slot_;
    if (P.events.empty()) {
        hipEvent_t e;
        // timing-only events: no system-scope fence, so no cache writeback in the interval
        KHOP_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        P.events.push_back(e);
    }
    e0_ = P.events.back();
    P.events.pop_back();
    prof_delay(st_);
    KHOP_HIP(hipEventRecord(e0_, st_));
}

void ProfScope::end(double fixed_bytes, double w0, double w1, double w2, double w3) {
    if (!e0_) return;
    Profiler &P = g_->prof;
    std::lock_guard<std::mutex> lk(g_->prof_mu);
    if (P.events.empty()) {
        hipEvent_t e;
        // timing-only events: no system-scope fence, so no cache writeback in the interval
        KHOP_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        P.events.push_back(e);
    }
    hipEvent_t e1 = P.events.back();
    P.events.pop_back();
    KHOP_HIP(hipEventRecord(e1, st_));
    P.pending.push_back({kind_, e0_, e1, fixed_bytes, slot_, {w0, w1, w2, w3}, -1, 0});
    e0_ = nullptr;
}

void ProfScope::end_split(double fixed_bytes, double w0, int alt_kind, int alt_field) {
    if (!e0_) return;
    end(fixed_bytes, w0);
    std::lock_guard<std::mutex> lk(g_->prof_mu);
    Profiler::Pending &p = g_->prof.pending.back();
    p.alt_kind = alt_kind;
    p.alt_field = alt_field;
}

// Waits for every pending profiled launch and folds it into the totals.
void prof_collect(khop_graph *g) {
    Profiler &P = g->prof;
    if (P.pending.empty()) return;
    constexpr int kLanes = 64;  // per-field lanes the kernels spread their counter atomics over
    std::vector<int64_t> units((size_t)P.next_slot * 4 * kLanes, 0);
    KHOP_HIP(hipEventSynchronize(P.pending.back().e1));
    for (auto &p : P.pending) KHOP_HIP(hipEventSynchronize(p.e1));
    if (P.next_slot > 0)
        KHOP_HIP(hipMemcpy(units.data(), P.d_units, units.size() * 8, hipMemcpyDeviceToHost));
    for (auto &p : P.pending) {
        float ms = 0;
        KHOP_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
        double bytes = p.fixed_bytes;
        int64_t field[4] = {0, 0, 0, 0};
        if (p.slot >= 0)
            for (int i = 0; i < 4; ++i) {
                for (int l = 0; l < kLanes; ++l) field[i] += units[((size_t)p.slot * 4 + i) * kLanes + l];
                bytes += p.w[i] * (double)field[i];
            }
        const int kind = (p.alt_kind >= 0 && field[p.alt_field] != 0) ? p.alt_kind : p.kind;
        P.launches[kind] += 1;
        P.ms[kind] += ms;
        P.bytes[kind] += bytes;
        P.events.push_back(p.e0);
        P.events.push_back(p.e1);
    }
    P.pending.clear();
    if (P.next_slot > 0) KHOP_HIP(hipMemset(P.d_units, 0, (size_t)P.next_slot * 4 * kLanes * 8));
    P.next_slot = 0;
}

// ---------------------------------------------------------------- context pools

struct PlainSlot {
    PlainCtx *ctx;
    CtxUse use;
};
struct BatchSlot {
    BatchCtx *ctx;
    CtxUse use;
};

}  // namespace khop

using namespace khop;

// Per-graph pools live beside the graph (allocated on first use).
namespace khop {
struct Pools {
    std::vector<PlainSlot> plain;
    std::vector<BatchSlot> batch;
    // host-API device buffers, grown on demand, one set per concurrent host call
    struct Buffers {
        int32_t *d_seeds = nullptr;
        int64_t *d_counts = nullptr;
        int64_t *d_te = nullptr;
        int64_t cap = 0;
        int64_t *h_pinned = nullptr;  // 2 int64 for per-query readback
        int32_t *d_dist = nullptr;    // breadth-first distances (n), then the depth
        int64_t dist_cap = 0;
        uint64_t *d_label = nullptr;  // a vertex mask (ceil(n / 64) words)
        int64_t label_cap = 0;
    };
    std::vector<Buffers *> bufs;
};
static std::mutex g_pools_mu;
static std::vector<std::pair<khop_graph *, Pools *>> g_pools;

static Pools *pools_of(khop_graph *g) {
    std::lock_guard<std::mutex> lk(g_pools_mu);
    for (auto &p : g_pools)
        if (p.first == g) return p.second;
    Pools *p = new Pools();
    g_pools.push_back({g, p});
    return p;
}

static void pools_drop(khop_graph *g) {
    Pools *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pools_mu);
        for (size_t i = 0; i < g_pools.size(); ++i)
            if (g_pools[i].first == g) {
                p = g_pools[i].second;
                g_pools.erase(g_pools.begin() + (long)i);
                break;
            }
    }
    if (!p) return;
    for (auto &s : p->plain) {
        if (s.use.done) {
            (void)hipEventSynchronize(s.use.done);
            (void)hipEventDestroy(s.use.done);
        }
        plain_ctx_destroy(s.ctx);
    }
    for (auto &s : p->batch) {
        if (s.use.done) {
            (void)hipEventSynchronize(s.use.done);
            (void)hipEventDestroy(s.use.done);
        }
        batch_ctx_destroy(s.ctx);
    }
    for (auto *b : p->bufs) {
        (void)hipFree(b->d_seeds);
        (void)hipFree(b->d_counts);
        (void)hipFree(b->d_te);
        (void)hipFree(b->d_dist);
        (void)hipFree(b->d_label);
        if (b->h_pinned) (void)hipHostFree(b->h_pinned);
        delete b;
    }
    delete p;
}

// Takes a free context; work already queued on it from another stream is
// ordered before the new use by a device-side wait (no host block).
static PlainSlot take_plain(khop_graph *g, hipStream_t st) {
    Pools *p = pools_of(g);
    PlainSlot s{nullptr, {}};
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!p->plain.empty()) {
            s = p->plain.back();
            p->plain.pop_back();
        }
    }
    if (!s.ctx) {
        s.ctx = plain_ctx_create(g);
        KHOP_HIP(hipEventCreateWithFlags(&s.use.done, hipEventDisableTiming));
    } else if (s.use.stream != st) {
        KHOP_HIP(hipStreamWaitEvent(st, s.use.done, 0));
    }
    return s;
}

static void give_plain(khop_graph *g, PlainSlot s, hipStream_t st) {
    s.use.stream = st;
    KHOP_HIP(hipEventRecord(s.use.done, st));
    Pools *p = pools_of(g);
    std::lock_guard<std::mutex> lk(g->mu);
    p->plain.push_back(s);
}

static BatchSlot take_batch(khop_graph *g, int words, hipStream_t st) {
    Pools *p = pools_of(g);
    BatchSlot s{nullptr, {}};
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (size_t i = 0; i < p->batch.size(); ++i)
            if (batch_ctx_words(p->batch[i].ctx) == words) {
                s = p->batch[i];
                p->batch.erase(p->batch.begin() + (long)i);
                break;
            }
    }
    if (!s.ctx) {
        s.ctx = batch_ctx_create(g, words);
        KHOP_HIP(hipEventCreateWithFlags(&s.use.done, hipEventDisableTiming));
    } else if (s.use.stream != st) {
        KHOP_HIP(hipStreamWaitEvent(st, s.use.done, 0));
    }
    return s;
}

static void give_batch(khop_graph *g, BatchSlot s, hipStream_t st) {
    s.use.stream = st;
    KHOP_HIP(hipEventRecord(s.use.done, st));
    Pools *p = pools_of(g);
    std::lock_guard<std::mutex> lk(g->mu);
    p->batch.push_back(s);
}

static Pools::Buffers *take_buffers(khop_graph *g, int64_t need) {
    Pools *p = pools_of(g);
    Pools::Buffers *b = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!p->bufs.empty()) {
            b = p->bufs.back();
            p->bufs.pop_back();
        }
    }
    if (!b) {
        b = new Pools::Buffers();
        KHOP_HIP(hipHostMalloc((void **)&b->h_pinned, 2 * sizeof(int64_t), hipHostMallocDefault));
    }
    if (b->cap < need) {
        (void)hipFree(b->d_seeds);
        (void)hipFree(b->d_counts);
        (void)hipFree(b->d_te);
        b->d_seeds = nullptr;
        b->d_counts = b->d_te = nullptr;
        b->cap = 0;
        const int64_t cap = std::max<int64_t>(need, 1024);
        if (hipMalloc(&b->d_seeds, cap * 4) != hipSuccess || hipMalloc(&b->d_counts, cap * 8) != hipSuccess ||
            hipMalloc(&b->d_te, cap * 8) != hipSuccess) {
            (void)hipGetLastError();
            fail(KHOP_ENOMEM, "device allocation for query buffers failed");
        }
        b->cap = cap;
    }
    return b;
}

// Grows the distance buffer to n + 1 int32 (the distances, then the depth).
static void ensure_dist(Pools::Buffers *b, int64_t n) {
    if (b->dist_cap >= n + 1) return;
    (void)hipFree(b->d_dist);
    b->d_dist = nullptr;
    b->dist_cap = 0;
    if (hipMalloc(&b->d_dist, (size_t)(n + 1) * 4) != hipSuccess) {
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation of a distance vector failed");
    }
    b->dist_cap = n + 1;
}

// Grows the vertex-mask buffer to `words` words.
static void ensure_label(Pools::Buffers *b, int64_t words) {
    if (b->label_cap >= words) return;
    (void)hipFree(b->d_label);
    b->d_label = nullptr;
    b->label_cap = 0;
    if (hipMalloc(&b->d_label, (size_t)words * 8) != hipSuccess) {
        (void)hipGetLastError();
        fail(KHOP_ENOMEM, "device allocation of a vertex mask failed");
    }
    b->label_cap = words;
}

static void give_buffers(khop_graph *g, Pools::Buffers *b) {
    Pools *p = pools_of(g);
    std::lock_guard<std::mutex> lk(g->mu);
    p->bufs.push_back(b);
}

static void validate_seeds(const khop_graph *g, const int32_t *seeds, int64_t num) {
    for (int64_t i = 0; i < num; ++i)
        if (seeds[i] < 0 || (int64_t)seeds[i] >= g->n)
            fail(KHOP_EINVAL, "seed " + std::to_string(seeds[i]) + " at index " + std::to_string(i) +
                                  " is outside [0, " + std::to_string(g->n) + ")");
}

// Runs a sorted batch plan: slots grouped in launches of at most `per` seeds.
void run_batched(khop_graph *g, const int32_t *d_seeds, const int32_t *h_ks, int64_t num,
                        int64_t *d_counts, hipStream_t st, const uint64_t *d_vmask) {
    // by k, largest first, except that one-hop queries go last: they take no
    // bit (a launch answers them from their seeds' rows)
    const std::vector<int32_t> order = batch_order(h_ks, num);
    const int per = std::max(64, std::min(1024, params_of(g).batch_seeds));
    for (int64_t at = 0; at < num; at += per) {
        const int64_t cnt = std::min<int64_t>(per, num - at);
        const int words = (int)((cnt + 63) / 64);  // exact: unused words would only widen every gather
        std::vector<int32_t> ks((size_t)cnt);
        for (int64_t j = 0; j < cnt; ++j) ks[j] = h_ks[order[at + j]];
        BatchSlot s = take_batch(g, words, st);
        try {
            batch_run(g, s.ctx, d_seeds, order.data() + at, ks.data(), cnt, d_counts, st, d_vmask);
        } catch (...) {
            give_batch(g, s, st);
            throw;
        }
        give_batch(g, s, st);
    }
}

}  // namespace khop

// ================================================================ C ABI

extern "C" {

const char *khop_last_error(void) { return t_err.c_str(); }

const char *khop_version(void) {
    static const std::string v = std::string("khop-mi355x 0.2 (gfx950, sources ") + source_hash() + ")";
    return v.c_str();
}

}  // extern "C"

// Builds a device graph from tuples (the body of graph_load_csr; throws khop::Error).
static void load_csr(const int32_t *src, const int32_t *dst, int64_t num_edges, int64_t num_vertices, uint32_t flags,
                     khop_graph **out) {
    if (!out) fail(KHOP_EINVAL, "out is NULL");
    if (num_edges < 0) fail(KHOP_EINVAL, "num_edges < 0");
    if (num_edges > 0 && (!src || !dst)) fail(KHOP_EINVAL, "src or dst is NULL with num_edges > 0");
    if (num_vertices <= 0) fail(KHOP_EINVAL, "num_vertices must be positive");
    if (num_vertices > INT32_MAX) fail(KHOP_ERANGE, "num_vertices exceeds INT32_MAX (int32 column indices)");
    if (flags != KHOP_UNDIRECTED && flags != KHOP_DIRECTED) fail(KHOP_EINVAL, "unknown flags");
    if (num_edges > ((int64_t)1 << 61)) fail(KHOP_ERANGE, "too many edges");
    // endpoint range check, in parallel
    {
        const int T = host_threads();
        std::vector<int64_t> bad((size_t)T, -1);
        std::vector<std::thread> pool;
        for (int t = 0; t < T; ++t)
            pool.emplace_back([&, t] {
                const int64_t lo = num_edges * t / T, hi = num_edges * (t + 1) / T;
                for (int64_t i = lo; i < hi; ++i)
                    if (src[i] < 0 || src[i] >= num_vertices || dst[i] < 0 || dst[i] >= num_vertices) {
                        bad[(size_t)t] = i;
                        return;
                    }
            });
        for (auto &th : pool) th.join();
        for (int64_t b : bad)
            if (b >= 0)
                fail(KHOP_EINVAL, "edge " + std::to_string(b) + " has an endpoint outside [0, " +
                                      std::to_string(num_vertices) + ")");
    }
    const int dev = require_device();
    KHOP_HIP(hipSetDevice(dev));
    const bool directed = flags == KHOP_DIRECTED;
    HostCSR out_csr = build_csr(src, dst, num_edges, num_vertices, !directed);
    HostCSR in_csr;
    if (directed) in_csr = build_csr(dst, src, num_edges, num_vertices, false);
    // per-hop counters pack a degree sum into 33 bits
    if ((int64_t)out_csr.colidx.size() >= ((int64_t)1 << 33))
        fail(KHOP_ERANGE, "more than 2^33 stored arcs");
    auto *g = new khop_graph();
    g->device = dev;
    g->n = num_vertices;
    g->nnz = (int64_t)out_csr.colidx.size();
    g->directed = directed ? 1 : 0;
    g->hash = csr_hash(out_csr);
    {
        hipDeviceProp_t p;
        KHOP_HIP(hipGetDeviceProperties(&p, dev));
        g->cu_count = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
    }
    g->h_outdeg.resize((size_t)g->n);
    for (int64_t v = 0; v < g->n; ++v) g->h_outdeg[v] = out_csr.rowptr[v + 1] - out_csr.rowptr[v];
    if (directed) {
        g->h_indeg.resize((size_t)g->n);
        for (int64_t v = 0; v < g->n; ++v) g->h_indeg[v] = in_csr.rowptr[v + 1] - in_csr.rowptr[v];
    } else {
        g->h_indeg = g->h_outdeg;
    }
    // column arrays carry kColidxPad zero entries past the end: the kernels
    // read a lane's next four in-edges with one 16-byte load
    auto upload = [&](const HostCSR &c, int64_t **rp, int32_t **ci) {
        const size_t ncol = c.colidx.size() + (size_t)khop::kColidxPad;
        if (hipMalloc(rp, (c.rowptr.size()) * 8) != hipSuccess || hipMalloc(ci, ncol * 4) != hipSuccess) {
            (void)hipGetLastError();
            fail(KHOP_ENOMEM, "device allocation for the CSR failed");
        }
        KHOP_HIP(hipMemcpy(*rp, c.rowptr.data(), c.rowptr.size() * 8, hipMemcpyHostToDevice));
        if (!c.colidx.empty())
            KHOP_HIP(hipMemcpy(*ci, c.colidx.data(), c.colidx.size() * 4, hipMemcpyHostToDevice));
        KHOP_HIP(hipMemset(*ci + c.colidx.size(), 0, (size_t)khop::kColidxPad * 4));
    };
    // Each in-row starts with its four in-neighbors of largest out-degree
    // (ties: the lowest id), in that order, the rest following in ascending
    // order: a bottom-up scan that stops at its first frontier in-neighbor
    // meets the likeliest ones first.  The first of them is the vertex's
    // probe (-1: no in-edge).  Threads take vertex ranges.
    std::vector<int32_t> probe((size_t)g->n, -1);
    {
        HostCSR &in = directed ? in_csr : out_csr;
        const int T = host_threads();
        std::vector<std::thread> pool;
        for (int t = 0; t < T; ++t)
            pool.emplace_back([&, t] {
                constexpr int kTop = 4;
                std::vector<int32_t> rest;
                const int64_t lo = g->n * t / T, hi = g->n * (t + 1) / T;
                for (int64_t v = lo; v < hi; ++v) {
                    int32_t *row = in.colidx.data() + in.rowptr[v];
                    const int64_t d = in.rowptr[v + 1] - in.rowptr[v];
                    if (d == 0) continue;
                    int64_t top[kTop];  // positions in the row, best first
                    int nt = 0;
                    for (int64_t x = 0; x < d; ++x) {
                        const int64_t od = g->h_outdeg[row[x]];
                        int j = nt;  // ascending ids: a later entry wins only with a larger degree
                        while (j > 0 && g->h_outdeg[row[top[j - 1]]] < od) --j;
                        if (j >= kTop) continue;
                        for (int q = std::min(nt, kTop - 1); q > j; --q) top[q] = top[q - 1];
                        top[j] = x;
                        nt = std::min(nt + 1, kTop);
                    }
                    rest.clear();
                    int32_t first[kTop];
                    for (int q = 0; q < nt; ++q) first[q] = row[top[q]];
                    for (int64_t x = 0; x < d; ++x) {
                        bool chosen = false;
                        for (int q = 0; q < nt; ++q) chosen |= top[q] == x;
                        if (!chosen) rest.push_back(row[x]);
                    }
                    std::copy(first, first + nt, row);
                    std::copy(rest.begin(), rest.end(), row + nt);
                    probe[(size_t)v] = row[0];
                }
            });
        for (auto &th : pool) th.join();
    }
    try {
        if (hipMalloc(&g->d_probe, (size_t)g->n * 4) != hipSuccess) {
            (void)hipGetLastError();
            fail(KHOP_ENOMEM, "device allocation for the probe in-neighbors failed");
        }
        KHOP_HIP(hipMemcpy(g->d_probe, probe.data(), (size_t)g->n * 4, hipMemcpyHostToDevice));
        upload(out_csr, &g->d_rowptr, &g->d_colidx);
        if (directed) {
            upload(in_csr, &g->d_in_rowptr, &g->d_in_colidx);
        } else {
            g->d_in_rowptr = g->d_rowptr;
            g->d_in_colidx = g->d_colidx;
        }
        KHOP_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        // the bottom-up chunk table for the default threshold, so that a path
        // which may not allocate finds one
        (void)plain_heavy_table(g, g->params.pull_heavy);
    } catch (...) {
        graph_free(g);
        throw;
    }
    *out = g;
    }

extern "C" {

int graph_load_csr(const int32_t *src, const int32_t *dst, int64_t num_edges, int64_t num_vertices, uint32_t flags,
                   khop_graph **out) {
    return guard([&] {
        load_csr(src, dst, num_edges, num_vertices, flags, out);
    });
}

int graph_load_csr_typed(const int32_t *src, const int32_t *dst, const uint8_t *rel, int64_t num_edges,
                         int64_t num_vertices, uint32_t flags, uint64_t rel_mask, khop_graph **out) {
    return guard([&] {
        if (num_edges < 0) fail(KHOP_EINVAL, "num_edges < 0");
        if (num_edges > 0 && (!src || !dst || !rel)) fail(KHOP_EINVAL, "src, dst or rel is NULL with num_edges > 0");
        // the union of the selected relations' adjacency matrices: the tuples of those relations
        std::vector<int32_t> fs, fd;
        fs.reserve((size_t)num_edges);
        fd.reserve((size_t)num_edges);
        for (int64_t i = 0; i < num_edges; ++i) {
            if (rel[i] >= 64)
                fail(KHOP_EINVAL, "relation type " + std::to_string(rel[i]) + " at index " + std::to_string(i) +
                                      " is not below 64");
            if ((rel_mask >> rel[i]) & 1ull) {
                fs.push_back(src[i]);
                fd.push_back(dst[i]);
            }
        }
        load_csr(fs.data(), fd.data(), (int64_t)fs.size(), num_vertices, flags, out);
    });
}

int graph_free(khop_graph *g) {
    return guard([&] {
        if (!g) return;
        (void)hipSetDevice(g->device);
        (void)hipDeviceSynchronize();
        pools_drop(g);
        if (g->d_in_rowptr && g->d_in_rowptr != g->d_rowptr) (void)hipFree(g->d_in_rowptr);
        if (g->d_in_colidx && g->d_in_colidx != g->d_colidx) (void)hipFree(g->d_in_colidx);
        if (g->d_rowptr) (void)hipFree(g->d_rowptr);
        if (g->d_colidx) (void)hipFree(g->d_colidx);
        if (g->d_probe) (void)hipFree(g->d_probe);
        heavy_tables_free(g);
        if (g->prof.d_units) (void)hipFree(g->prof.d_units);
        for (auto e : g->prof.events) (void)hipEventDestroy(e);
        if (g->stream) (void)hipStreamDestroy(g->stream);
        delete g;
    });
}

int graph_info(const khop_graph *g, int64_t *num_vertices, int64_t *num_arcs, int32_t *directed) {
    return guard([&] {
        check_graph(g);
        if (num_vertices) *num_vertices = g->n;
        if (num_arcs) *num_arcs = g->nnz;
        if (directed) *directed = g->directed;
    });
}

int graph_degrees(const khop_graph *g, int64_t *deg) {
    return guard([&] {
        check_graph(g);
        if (!deg) fail(KHOP_EINVAL, "deg is NULL");
        std::memcpy(deg, g->h_outdeg.data(), (size_t)g->n * 8);
    });
}

int khop_count(khop_graph *g, const int32_t *seeds, int64_t num_seeds, int32_t k, int64_t *counts,
               int64_t *traversed_edges) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        if (num_seeds == 0) return;
        if (!seeds || !counts) fail(KHOP_EINVAL, "seeds or counts is NULL");
        validate_seeds(g, seeds, num_seeds);
        if (k == 0) {
            std::fill(counts, counts + num_seeds, 0);
            if (traversed_edges) std::fill(traversed_edges, traversed_edges + num_seeds, 0);
            return;
        }
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        Pools::Buffers *b = take_buffers(g, num_seeds);
        PlainSlot s{nullptr, {}};
        std::vector<int64_t> c((size_t)num_seeds), t((size_t)num_seeds);
        try {
            KHOP_HIP(hipMemcpyAsync(b->d_seeds, seeds, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
            s = take_plain(g, st);
            for (int64_t i = 0; i < num_seeds; ++i) {
                plain_run(g, s.ctx, b->d_seeds + i, 1, k, b->d_counts + i, b->d_te + i, st);
                KHOP_HIP(hipMemcpyAsync(b->h_pinned, b->d_counts + i, 8, hipMemcpyDeviceToHost, st));
                KHOP_HIP(hipMemcpyAsync(b->h_pinned + 1, b->d_te + i, 8, hipMemcpyDeviceToHost, st));
                KHOP_HIP(hipStreamSynchronize(st));
                c[i] = b->h_pinned[0];
                t[i] = b->h_pinned[1];
            }
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        give_buffers(g, b);
        std::copy(c.begin(), c.end(), counts);
        if (traversed_edges) std::copy(t.begin(), t.end(), traversed_edges);
    });
}

int khop_count_dev(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                   int64_t *d_traversed_edges, void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        if (num_seeds == 0) return;
        if (!d_seeds || !d_counts) fail(KHOP_EINVAL, "d_seeds or d_counts is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        if (k == 0) {
            plain_fill_zero_outputs(d_counts, d_traversed_edges, num_seeds, st);
            return;
        }
        PlainSlot s = take_plain(g, st);
        try {
            plain_run(g, s.ctx, d_seeds, num_seeds, k, d_counts, d_traversed_edges, st);
        } catch (...) {
            give_plain(g, s, st);
            throw;
        }
        give_plain(g, s, st);
    });
}

int khop_count_dev_noalloc(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k, int64_t *d_counts,
                           int64_t *d_traversed_edges, void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        if (num_seeds == 0) return;
        if (!d_seeds || !d_counts) fail(KHOP_EINVAL, "d_seeds or d_counts is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        plain_run_noalloc(g, d_seeds, num_seeds, k, d_counts, d_traversed_edges, (hipStream_t)hip_stream);
    });
}

int khop_count_labeled(khop_graph *g, const int32_t *seeds, int64_t num_seeds, int32_t k, const uint64_t *label_bits,
                       int64_t *counts, int64_t *traversed_edges) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        if (num_seeds == 0) return;
        if (!seeds || !counts || !label_bits) fail(KHOP_EINVAL, "seeds, counts or label_bits is NULL");
        validate_seeds(g, seeds, num_seeds);
        if (k == 0) {
            std::fill(counts, counts + num_seeds, 0);
            if (traversed_edges) std::fill(traversed_edges, traversed_edges + num_seeds, 0);
            return;
        }
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        const int64_t words = (g->n + 63) / 64;
        Pools::Buffers *b = take_buffers(g, num_seeds);
        PlainSlot s{nullptr, {}};
        std::vector<int64_t> c((size_t)num_seeds), t((size_t)num_seeds);
        try {
            ensure_label(b, words);
            KHOP_HIP(hipMemcpyAsync(b->d_label, label_bits, (size_t)words * 8, hipMemcpyHostToDevice, st));
            KHOP_HIP(hipMemcpyAsync(b->d_seeds, seeds, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
            s = take_plain(g, st);
            plain_run(g, s.ctx, b->d_seeds, num_seeds, k, b->d_counts, b->d_te, st, b->d_label);
            KHOP_HIP(hipMemcpyAsync(c.data(), b->d_counts, (size_t)num_seeds * 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipMemcpyAsync(t.data(), b->d_te, (size_t)num_seeds * 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        give_buffers(g, b);
        std::copy(c.begin(), c.end(), counts);
        if (traversed_edges) std::copy(t.begin(), t.end(), traversed_edges);
    });
}

int khop_count_labeled_dev(khop_graph *g, const int32_t *d_seeds, int64_t num_seeds, int32_t k,
                           const uint64_t *d_label_bits, int64_t *d_counts, int64_t *d_traversed_edges,
                           void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        if (num_seeds == 0) return;
        if (!d_seeds || !d_counts || !d_label_bits) fail(KHOP_EINVAL, "d_seeds, d_counts or d_label_bits is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        if (k == 0) {
            plain_fill_zero_outputs(d_counts, d_traversed_edges, num_seeds, st);
            return;
        }
        PlainSlot s = take_plain(g, st);
        try {
            plain_run(g, s.ctx, d_seeds, num_seeds, k, d_counts, d_traversed_edges, st, d_label_bits);
        } catch (...) {
            give_plain(g, s, st);
            throw;
        }
        give_plain(g, s, st);
    });
}

int khop_count_batched(khop_graph *g, const int32_t *seeds, const int32_t *ks, int64_t num_seeds, int64_t *counts) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (num_seeds == 0) return;
        if (!seeds || !ks || !counts) fail(KHOP_EINVAL, "seeds, ks or counts is NULL");
        validate_seeds(g, seeds, num_seeds);
        for (int64_t i = 0; i < num_seeds; ++i)
            if (ks[i] < 0) fail(KHOP_EINVAL, "k < 0 at index " + std::to_string(i));
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        Pools::Buffers *b = take_buffers(g, num_seeds);
        std::vector<int64_t> c((size_t)num_seeds);
        try {
            KHOP_HIP(hipMemcpyAsync(b->d_seeds, seeds, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
            run_batched(g, b->d_seeds, ks, num_seeds, b->d_counts, st);
            KHOP_HIP(hipMemcpyAsync(c.data(), b->d_counts, (size_t)num_seeds * 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
        } catch (...) {
            give_buffers(g, b);
            throw;
        }
        give_buffers(g, b);
        std::copy(c.begin(), c.end(), counts);
    });
}

int khop_count_batched_dev(khop_graph *g, const int32_t *d_seeds, const int32_t *d_ks, int64_t num_seeds,
                           int64_t *d_counts, void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (num_seeds == 0) return;
        if (!d_seeds || !d_ks || !d_counts) fail(KHOP_EINVAL, "d_seeds, d_ks or d_counts is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        // the level plan (seed order by k, active masks) is made on the host
        std::vector<int32_t> hs((size_t)num_seeds), hk((size_t)num_seeds);
        KHOP_HIP(hipMemcpyAsync(hs.data(), d_seeds, (size_t)num_seeds * 4, hipMemcpyDeviceToHost, st));
        KHOP_HIP(hipMemcpyAsync(hk.data(), d_ks, (size_t)num_seeds * 4, hipMemcpyDeviceToHost, st));
        KHOP_HIP(hipStreamSynchronize(st));
        validate_seeds(g, hs.data(), num_seeds);
        for (int64_t i = 0; i < num_seeds; ++i)
            if (hk[i] < 0) fail(KHOP_EINVAL, "k < 0 at index " + std::to_string(i));
        run_batched(g, d_seeds, hk.data(), num_seeds, d_counts, st);
    });
}

int khop_bfs(khop_graph *g, int32_t seed, int32_t max_depth, int32_t *dist, int64_t *count, int32_t *depth) {
    return guard([&] {
        check_graph(g);
        if (!dist) fail(KHOP_EINVAL, "dist is NULL");
        validate_seeds(g, &seed, 1);
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        Pools::Buffers *b = take_buffers(g, 1);
        PlainSlot s{nullptr, {}};
        int64_t c = 0;
        int32_t d = 0;
        try {
            ensure_dist(b, g->n);
            s = take_plain(g, st);
            plain_bfs(g, s.ctx, seed, max_depth, b->d_dist, b->d_counts, b->d_dist + g->n, nullptr, 0,
                      (int32_t *)b->h_pinned, st);
            KHOP_HIP(hipMemcpyAsync(dist, b->d_dist, (size_t)g->n * 4, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipMemcpyAsync(b->h_pinned, b->d_counts, 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipMemcpyAsync(b->h_pinned + 1, b->d_dist + g->n, 4, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
            c = b->h_pinned[0];
            d = *(const int32_t *)(b->h_pinned + 1);
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        give_buffers(g, b);
        if (count) *count = c;
        if (depth) *depth = d;
    });
}

int khop_bfs_dev(khop_graph *g, int32_t seed, int32_t max_depth, int32_t *d_dist, int64_t *d_count, int32_t *d_depth,
                 void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (!d_dist) fail(KHOP_EINVAL, "d_dist is NULL");
        validate_seeds(g, &seed, 1);
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        Pools::Buffers *b = max_depth < 0 ? take_buffers(g, 1) : nullptr;
        PlainSlot s{nullptr, {}};
        try {
            s = take_plain(g, st);
            plain_bfs(g, s.ctx, seed, max_depth, d_dist, d_count, d_depth, nullptr, 0,
                      b ? (int32_t *)b->h_pinned : nullptr, st);
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            if (b) give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        if (b) give_buffers(g, b);
    });
}

int khop_levels(khop_graph *g, int32_t seed, int32_t k, int64_t *level_counts) {
    return guard([&] {
        check_graph(g);
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        validate_seeds(g, &seed, 1);
        if (k == 0) return;
        if (!level_counts) fail(KHOP_EINVAL, "level_counts is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        Pools::Buffers *b = take_buffers(g, k);
        PlainSlot s{nullptr, {}};
        std::vector<int64_t> lv((size_t)k);
        try {
            s = take_plain(g, st);
            plain_bfs(g, s.ctx, seed, k, nullptr, nullptr, nullptr, b->d_counts, k, (int32_t *)b->h_pinned, st);
            KHOP_HIP(hipMemcpyAsync(lv.data(), b->d_counts, (size_t)k * 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        give_buffers(g, b);
        std::copy(lv.begin(), lv.end(), level_counts);
    });
}

int khop_levels_dev(khop_graph *g, int32_t seed, int32_t k, int64_t *d_level_counts, void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (k < 0) fail(KHOP_EINVAL, "k < 0");
        validate_seeds(g, &seed, 1);
        if (k == 0) return;
        if (!d_level_counts) fail(KHOP_EINVAL, "d_level_counts is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        PlainSlot s = take_plain(g, st);
        try {
            plain_bfs(g, s.ctx, seed, k, nullptr, nullptr, nullptr, d_level_counts, k, nullptr, st);
        } catch (...) {
            give_plain(g, s, st);
            throw;
        }
        give_plain(g, s, st);
    });
}

int khop_neighborhood(khop_graph *g, int32_t seed, int32_t k, int32_t *ids, int64_t capacity, int64_t *count) {
    return guard([&] {
        check_graph(g);
        if (capacity < 0) fail(KHOP_EINVAL, "capacity < 0");
        if (capacity > 0 && !ids) fail(KHOP_EINVAL, "ids is NULL with capacity > 0");
        if (!count) fail(KHOP_EINVAL, "count is NULL");
        validate_seeds(g, &seed, 1);
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        Pools::Buffers *b = take_buffers(g, 1);
        PlainSlot s{nullptr, {}};
        int64_t c = 0;
        const int64_t cap = std::min<int64_t>(capacity, g->n);
        try {
            ensure_dist(b, g->n);
            s = take_plain(g, st);
            plain_bfs(g, s.ctx, seed, k, nullptr, nullptr, nullptr, nullptr, 0, (int32_t *)b->h_pinned, st);
            plain_set(g, s.ctx, seed, b->d_dist, cap, b->d_counts, st);
            KHOP_HIP(hipMemcpyAsync(b->h_pinned, b->d_counts, 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
            c = b->h_pinned[0];
            const int64_t m = std::min(c, cap);
            if (m > 0) {
                KHOP_HIP(hipMemcpyAsync(ids, b->d_dist, (size_t)m * 4, hipMemcpyDeviceToHost, st));
                KHOP_HIP(hipStreamSynchronize(st));
            }
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        give_buffers(g, b);
        *count = c;
    });
}

int khop_neighborhood_dev(khop_graph *g, int32_t seed, int32_t k, int32_t *d_ids, int64_t capacity, int64_t *d_count,
                          void *hip_stream) {
    return guard([&] {
        check_graph(g);
        if (capacity < 0) fail(KHOP_EINVAL, "capacity < 0");
        if (capacity > 0 && !d_ids) fail(KHOP_EINVAL, "d_ids is NULL with capacity > 0");
        if (!d_count) fail(KHOP_EINVAL, "d_count is NULL");
        validate_seeds(g, &seed, 1);
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = (hipStream_t)hip_stream;
        Pools::Buffers *b = k < 0 ? take_buffers(g, 1) : nullptr;
        PlainSlot s{nullptr, {}};
        try {
            s = take_plain(g, st);
            plain_bfs(g, s.ctx, seed, k, nullptr, nullptr, nullptr, nullptr, 0, b ? (int32_t *)b->h_pinned : nullptr,
                      st);
            plain_set(g, s.ctx, seed, d_ids, std::min<int64_t>(capacity, g->n), d_count, st);
        } catch (...) {
            if (s.ctx) give_plain(g, s, st);
            if (b) give_buffers(g, b);
            throw;
        }
        give_plain(g, s, st);
        if (b) give_buffers(g, b);
    });
}

int khop_count_batched_labeled(khop_graph *g, const int32_t *seeds, const int32_t *ks, int64_t num_seeds,
                               const uint64_t *label_bits, int64_t *counts) {
    return guard([&] {
        check_graph(g);
        if (num_seeds < 0) fail(KHOP_EINVAL, "num_seeds < 0");
        if (num_seeds == 0) return;
        if (!seeds || !ks || !counts || !label_bits) fail(KHOP_EINVAL, "seeds, ks, counts or label_bits is NULL");
        validate_seeds(g, seeds, num_seeds);
        for (int64_t i = 0; i < num_seeds; ++i)
            if (ks[i] < 0) fail(KHOP_EINVAL, "k < 0 at index " + std::to_string(i));
        KHOP_HIP(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        const int64_t words = (g->n + 63) / 64;
        Pools::Buffers *b = take_buffers(g, num_seeds);
        std::vector<int64_t> c((size_t)num_seeds);
        try {
            ensure_label(b, words);
            KHOP_HIP(hipMemcpyAsync(b->d_label, label_bits, (size_t)words * 8, hipMemcpyHostToDevice, st));
            KHOP_HIP(hipMemcpyAsync(b->d_seeds, seeds, (size_t)num_seeds * 4, hipMemcpyHostToDevice, st));
            run_batched(g, b->d_seeds, ks, num_seeds, b->d_counts, st, b->d_label);
            KHOP_HIP(hipMemcpyAsync(c.data(), b->d_counts, (size_t)num_seeds * 8, hipMemcpyDeviceToHost, st));
            KHOP_HIP(hipStreamSynchronize(st));
        } catch (...) {
            give_buffers(g, b);
            throw;
        }
        give_buffers(g, b);
        std::copy(c.begin(), c.end(), counts);
    });
}

int khop_set_option(khop_graph *g, int32_t option, int64_t value) {
    return guard([&] {
        check_graph(g);
        std::lock_guard<std::mutex> lk(g->params_mu);
        Params &P = g->params;
        switch (option) {
            case KHOP_OPT_DIRECTION:
                if (value != KHOP_DIR_AUTO && value != KHOP_DIR_PUSH && value != KHOP_DIR_PULL)
                    fail(KHOP_EINVAL, "direction must be KHOP_DIR_AUTO, KHOP_DIR_PUSH or KHOP_DIR_PULL");
                P.dir_mode = (int)value;
                break;
            case KHOP_OPT_ALPHA:
                if (value < 1 || value > (1 << 20)) fail(KHOP_EINVAL, "alpha out of range [1, 2^20]");
                P.alpha = (int)value;
                break;
            case KHOP_OPT_BETA:
                if (value < 1 || value > (1 << 20)) fail(KHOP_EINVAL, "beta out of range [1, 2^20]");
                P.beta = (int)value;
                break;
            case KHOP_OPT_PULL_LIGHT:
                if (value < 0 || value > (1 << 20)) fail(KHOP_EINVAL, "pull light threshold out of range");
                P.pull_light = (int)value;
                break;
            case KHOP_OPT_BATCH_SEEDS:
                if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
                    fail(KHOP_EINVAL, "batch seeds must be 64, 128, 256, 512 or 1024");
                P.batch_seeds = (int)value;
                break;
            case KHOP_OPT_BATCH_HEAVY:
                if (value < 1 || value > INT32_MAX) fail(KHOP_EINVAL, "heavy threshold out of range");
                P.batch_heavy = (int)value;
                break;
            case KHOP_OPT_BATCH_PUSH:
                if (value < 1 || value > (1 << 30)) fail(KHOP_EINVAL, "batch push divisor out of range");
                P.batch_push_div = (int)value;
                break;
            case KHOP_OPT_PULL_HEAVY:
                if (value < 1 || value > INT32_MAX) fail(KHOP_EINVAL, "pull heavy threshold out of range [1, 2^31)");
                P.pull_heavy = (int)value;
                break;
            case KHOP_OPT_PUSH_ATOMIC:
                if (value < 0 || value > INT32_MAX) fail(KHOP_EINVAL, "push atomic limit out of range [0, 2^31)");
                P.push_atomic_max = (int)value;
                break;
            case KHOP_OPT_PLAIN_GRID:
                if (value < 1 || value > 64) fail(KHOP_EINVAL, "plain grid out of range [1, 64] blocks per CU");
                P.plain_grid = (int)value;
                break;
            case KHOP_OPT_BATCH_GRID:
                if (value < 1 || value > 64) fail(KHOP_EINVAL, "batch grid out of range [1, 64] blocks per CU");
                P.batch_grid = (int)value;
                break;
            case KHOP_OPT_PLAIN_PIPELINE:
                if (value != 0 && value != 1) fail(KHOP_EINVAL, "plain pipeline must be 0 or 1");
                P.plain_pipeline = (int)value;
                break;
            case KHOP_OPT_PLAIN_GRAPHS:
                if (value != 0 && value != 1) fail(KHOP_EINVAL, "plain graphs must be 0 or 1");
                P.plain_graphs = (int)value;
                break;
            default:
                fail(KHOP_EINVAL, "unknown option " + std::to_string(option));
        }
    });
}

int khop_get_option(const khop_graph *g, int32_t option, int64_t *value) {
    return guard([&] {
        check_graph(g);
        if (!value) fail(KHOP_EINVAL, "value is NULL");
        const Params P = params_of(const_cast<khop_graph *>(g));
        switch (option) {
            case KHOP_OPT_DIRECTION: *value = P.dir_mode; break;
            case KHOP_OPT_ALPHA: *value = P.alpha; break;
            case KHOP_OPT_BETA: *value = P.beta; break;
            case KHOP_OPT_PULL_LIGHT: *value = P.pull_light; break;
            case KHOP_OPT_BATCH_SEEDS: *value = P.batch_seeds; break;
            case KHOP_OPT_BATCH_HEAVY: *value = P.batch_heavy; break;
            case KHOP_OPT_BATCH_PUSH: *value = P.batch_push_div; break;
            case KHOP_OPT_PULL_HEAVY: *value = P.pull_heavy; break;
            case KHOP_OPT_PUSH_ATOMIC: *value = P.push_atomic_max; break;
            case KHOP_OPT_PLAIN_GRID: *value = P.plain_grid; break;
            case KHOP_OPT_BATCH_GRID: *value = P.batch_grid; break;
            case KHOP_OPT_PLAIN_PIPELINE: *value = P.plain_pipeline; break;
            case KHOP_OPT_PLAIN_GRAPHS: *value = P.plain_graphs; break;
            default: fail(KHOP_EINVAL, "unknown option " + std::to_string(option));
        }
    });
}

int khop_profile(khop_graph *g, int32_t enable) {
    return guard([&] {
        check_graph(g);
        KHOP_HIP(hipSetDevice(g->device));
        {
            std::lock_guard<std::mutex> lk(g->prof_mu);
            Profiler &P = g->prof;
            if (enable) {
                if (!P.d_units) {
                    P.cap = 1 << 15;  // launches per collection; 2 KiB of counters each
                    if (hipMalloc(&P.d_units, (size_t)P.cap * 4 * 64 * 8) != hipSuccess) {
                        (void)hipGetLastError();
                        P.d_units = nullptr;
                        fail(KHOP_ENOMEM, "device allocation for profiling counters failed");
                    }
                }
                prof_collect(g);
                KHOP_HIP(hipMemset(P.d_units, 0, (size_t)P.cap * 4 * 64 * 8));
                KHOP_HIP(hipDeviceSynchronize());
                P.next_slot = 0;
                std::fill(std::begin(P.launches), std::end(P.launches), 0);
                std::fill(std::begin(P.ms), std::end(P.ms), 0.0);
                std::fill(std::begin(P.bytes), std::end(P.bytes), 0.0);
                P.on = true;
            } else {
                prof_collect(g);
                P.on = false;
            }
        }
        if (enable) {
            // the cost of the measurement itself: empty launches bracketed like every profiled one
            hipStream_t st;
            KHOP_HIP(hipStreamCreate(&st));
            for (int i = 0; i < 16; ++i) {
                ProfScope ps(g, KK_EMPTY_LAUNCH, st);
                prof_empty(st);
                ps.end(0);
            }
            KHOP_HIP(hipStreamSynchronize(st));
            KHOP_HIP(hipStreamDestroy(st));
        }
    });
}

int khop_profile_read(khop_graph *g, khop_kernel_stat *out, int32_t max, int32_t *n_out) {
    return guard([&] {
        check_graph(g);
        if (!n_out || (max > 0 && !out)) fail(KHOP_EINVAL, "out or n_out is NULL");
        KHOP_HIP(hipSetDevice(g->device));
        std::lock_guard<std::mutex> lk(g->prof_mu);
        prof_collect(g);
        Profiler &P = g->prof;
        int32_t n = 0;
        for (int kk = 0; kk < KK_COUNT_KINDS; ++kk) {
            if (P.launches[kk] == 0) continue;
            if (n < max) {
                khop_kernel_stat &s = out[n];
                std::memset(&s, 0, sizeof(s));
                std::strncpy(s.name, kKernelNames[kk], sizeof(s.name) - 1);
                s.launches = P.launches[kk];
                s.total_ms = P.ms[kk];
                s.algorithmic_bytes = P.bytes[kk];
            }
            ++n;
        }
        *n_out = std::min(n, std::max(max, 0));
    });
}

}  // extern "C"
