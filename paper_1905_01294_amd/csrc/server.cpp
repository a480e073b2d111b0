// Continuous-batching server for k-hop queries.
//
// The paper serves many concurrent queries from a worker pool, one query per
// worker, arguing that throughput under concurrency matters more than the
// latency of one query on all cores (Section II).  The GPU analog here keeps
// every graph resident and answers queries through two kinds of lanes per
// graph (the rules are in serve_policy.h, where they can be checked without a
// GPU):
//   - two batch lanes, one for queries with k <= 2 and one for deeper ones,
//     so short queries never wait behind deep traversals.  Each lane has two
//     run slots, each with its own HIP stream.  A free slot takes what waits
//     in its lane (FIFO, up to 64 queries per word of its context) and
//     enqueues it as one batched launch sequence (batch_run: seeds as bit
//     columns of one bitset product per hop, one-hop queries from their
//     seeds' rows, finished seeds narrowed away); arrivals that come while
//     both slots run join the next launch the moment a slot frees.  So the
//     launches of a lane, and of all lanes and graphs, overlap on the device,
//     and the batch size follows the load.  A slot holds its batch context
//     only while it has work, sized by the memory budget left, so queries
//     wait rather than fail when memory is short;
//   - a single-query lane on a stream of its own, which runs queries one
//     after another through the plain path (the paper's one query per
//     worker), in groups of one k, and takes arrivals only while the device
//     time it would need stays low and it would answer before a batch lane.
// A scheduler thread runs the lanes: it turns completed launches into
// results, routes arrivals, and plans the next launches.
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <thread>

#include "khop_impl.h"
#include "serve_policy.h"

namespace {

using khop::ServeRequest;

int64_t mono_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

constexpr size_t kMaxQueued = 1 << 22;
constexpr int kPlainGroup = 64;  // queries of one k per plain launch sequence
constexpr int kCostBuckets = 17; // per-k cost estimates; k >= 16 share the last

// Counters of one lane, read by khop_server_stats (guarded by the server's mutex).
struct LaneStats {
    int64_t launches = 0, queries = 0;
    double busy_ms = 0, max_ms = 0;
    int32_t words = 0, queued = 0;
    void add(int64_t q, double ms) {
        launches += 1;
        queries += q;
        busy_ms += ms;
        max_ms = std::max(max_ms, ms);
    }
};

// Device side of one run slot of a batch lane.
struct RunRes {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    khop::BatchCtx *ctx = nullptr;
    int32_t *d_seeds = nullptr, *h_seeds = nullptr;  // 64 * max_words entries
    int64_t *d_counts = nullptr, *h_counts = nullptr;
};

struct BatchLane {
    khop_graph *g = nullptr;
    int graph_id = 0, lane = 0;
    khop::LanePlan plan;
    RunRes res[khop::kRunsPerLane];
    LaneStats stats;
};

// The single-query lane of one graph.
struct PlainLane {
    khop_graph *g = nullptr;
    int graph_id = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // timing only, around the launch sequence
    hipEvent_t ev_end = nullptr;                        // completion, after the counts' copy
    khop::PlainCtx *ctx = nullptr;
    int32_t *d_seeds = nullptr;  // kPlainGroup
    int64_t *d_counts = nullptr;
    int32_t *h_seeds = nullptr;  // pinned staging
    int64_t *h_counts = nullptr;
    std::deque<ServeRequest> queue;
    std::vector<ServeRequest> running;
    int64_t t_admit = 0;
    bool inflight = false;
    double cost_ms[kCostBuckets];   // moving average of one query's device time by k
    double floor_ms[kCostBuckets];  // the least per-query device time a group of that k took (uncontended)
    double backlog_ms = 0;          // expected device time of the queued and running queries
    LaneStats stats;
    PlainLane() {
        // optimistic until measured: the first queries are answered here and set the figures
        for (int k = 0; k < kCostBuckets; ++k) cost_ms[k] = floor_ms[k] = 0.005 * (k + 1);
    }
    double cost(int32_t k) const { return cost_ms[std::min<int32_t>(k, kCostBuckets - 1)]; }
    double floor_cost(int32_t k) const { return floor_ms[std::min<int32_t>(k, kCostBuckets - 1)]; }
};

}  // namespace

struct khop_server {
    int64_t budget = 0;
    int64_t used = 0;  // device bytes of the batch contexts held (scheduler thread only)
    int max_words = 16;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<BatchLane *> lanes;   // kServeLanes per graph, graph i's at [i * kServeLanes, ...)
    std::vector<PlainLane *> plains;  // one per graph
    int ngraphs = 0;
    std::atomic<int> route{KHOP_ROUTE_AUTO};
    khop::SingleRouter router;
    bool waiting_mem = false;  // some lane found no memory in the last pass
    std::deque<ServeRequest> incoming;
    std::deque<khop_result> done;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    std::thread th;
    std::string thread_error;
};

namespace {

void finish(khop_server *s, const ServeRequest &r, int status, int64_t count, int64_t t_admit,
            int path = KHOP_PATH_BATCH) {
    khop_result res{};
    res.ticket = r.ticket;
    res.status = status;
    res.graph_id = r.graph_id;
    res.seed = r.seed;
    res.k = r.k;
    res.count = count;
    res.t_submit_ns = r.t_submit;
    res.t_admit_ns = t_admit;
    res.t_done_ns = mono_ns();
    res.path = path;
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(res);
    s->completed += 1;
    s->cv_done.notify_all();
}

void finish_late(khop_server *s, const std::vector<ServeRequest> &late, int path) {
    for (const ServeRequest &r : late) finish(s, r, KHOP_ETIMEDOUT, -1, 0, path);
}

// Enqueues one batched launch of `batch` on slot i of the lane.
void launch_batch(BatchLane &L, int i, const std::vector<ServeRequest> &batch) {
    RunRes &R = L.res[i];
    const int64_t n = (int64_t)batch.size();
    std::vector<int32_t> ks((size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        R.h_seeds[j] = batch[j].seed;
        ks[j] = batch[j].k;
    }
    const std::vector<int32_t> perm = khop::batch_order(ks.data(), n);
    std::vector<int32_t> ks_sorted((size_t)n);
    for (int64_t j = 0; j < n; ++j) ks_sorted[j] = ks[perm[j]];
    KHOP_HIP(hipMemcpyAsync(R.d_seeds, R.h_seeds, (size_t)n * 4, hipMemcpyHostToDevice, R.stream));
    khop::batch_run(L.g, R.ctx, R.d_seeds, perm.data(), ks_sorted.data(), n, R.d_counts, R.stream);
    KHOP_HIP(hipMemcpyAsync(R.h_counts, R.d_counts, (size_t)n * 8, hipMemcpyDeviceToHost, R.stream));
    KHOP_HIP(hipEventRecord(R.done, R.stream));
}

// Completed launches of a lane become results.
bool poll_lane(khop_server *s, BatchLane &L, int64_t now) {
    bool busy = false;
    for (int i = 0; i < khop::kRunsPerLane; ++i) {
        khop::LanePlan::Run &r = L.plan.runs[i];
        if (!r.busy) continue;
        if (hipEventQuery(L.res[i].done) != hipSuccess) {
            busy = true;
            continue;
        }
        const int64_t *counts = L.res[i].h_counts;
        for (size_t j = 0; j < r.reqs.size(); ++j) finish(s, r.reqs[j], KHOP_OK, counts[j], r.t_launch);
        const double ms = (double)(now - r.t_launch) / 1e6;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            L.stats.add((int64_t)r.reqs.size(), ms);
        }
        khop::complete_run(L.plan, i, now);
    }
    return busy;
}

// Plans and enqueues a lane's next launches; returns whether it still has work.
bool plan_batch_lane(khop_server *s, BatchLane &L, int64_t now, int64_t &avail, bool &waiting) {
    const khop_graph *g = L.g;
    auto bytes_of = [g](int w) { return (int64_t)khop::batch_ctx_bytes(g->n, g->nnz, w); };
    khop::LaneActions a = khop::plan_lane(L.plan, now, avail, s->max_words, s->waiting_mem, bytes_of);
    for (int i : a.releases) {
        KHOP_HIP(hipStreamSynchronize(L.res[i].stream));
        khop::batch_ctx_destroy(L.res[i].ctx);
        L.res[i].ctx = nullptr;
    }
    finish_late(s, a.late, KHOP_PATH_BATCH);
    for (auto &ln : a.launches) {
        RunRes &R = L.res[ln.run];
        if (ln.alloc_words) {
            try {
                R.ctx = khop::batch_ctx_create(L.g, ln.alloc_words);
            } catch (const khop::Error &e) {
                if (e.status != KHOP_ENOMEM) throw;
                // the device had less free memory than the budget: wait, as for the budget
                khop::LanePlan::Run &r = L.plan.runs[ln.run];
                avail += r.bytes;
                r = khop::LanePlan::Run{};
                for (auto it = ln.batch.rbegin(); it != ln.batch.rend(); ++it) L.plan.queue.push_front(*it);
                a.waiting = true;
                continue;
            }
        }
        launch_batch(L, ln.run, ln.batch);
    }
    waiting |= a.waiting;
    int words = 0;
    for (auto &r : L.plan.runs) words = std::max(words, r.words);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        L.stats.words = words;
        L.stats.queued = (int32_t)std::min<size_t>(L.plan.queue.size(), INT32_MAX);
    }
    bool busy = !L.plan.queue.empty();
    for (auto &r : L.plan.runs) busy |= r.busy;
    return busy;
}

// Results of the plain group that just completed, and the cost estimate it updates.
void complete_plain(khop_server *s, PlainLane &pl) {
    float ms = 0;
    KHOP_HIP(hipEventElapsedTime(&ms, pl.ev_start, pl.ev_stop));
    const int m = (int)pl.running.size();
    const int32_t k = pl.running.front().k;
    const int b = std::min<int32_t>(k, kCostBuckets - 1);
    pl.cost_ms[b] = 0.7 * pl.cost_ms[b] + 0.3 * (double)ms / m;
    pl.floor_ms[b] = std::min(pl.floor_ms[b], (double)ms / m);
    for (int i = 0; i < m; ++i) {
        pl.backlog_ms = std::max(0.0, pl.backlog_ms - pl.running[i].plain_ms);
        finish(s, pl.running[i], KHOP_OK, pl.h_counts[i], pl.t_admit, KHOP_PATH_SINGLE);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        pl.stats.add(m, (double)(mono_ns() - pl.t_admit) / 1e6);
    }
    pl.running.clear();
}

// Starts the next plain group: the oldest queued query and up to kPlainGroup - 1
// more of the same k, one launch sequence.  Returns true if work was enqueued.
bool plan_plain(khop_server *s, PlainLane &pl, int64_t now) {
    for (auto it = pl.queue.begin(); it != pl.queue.end();) {
        if (khop::expired(*it, now)) {
            pl.backlog_ms = std::max(0.0, pl.backlog_ms - it->plain_ms);
            finish(s, *it, KHOP_ETIMEDOUT, -1, 0, KHOP_PATH_SINGLE);
            it = pl.queue.erase(it);
        } else {
            ++it;
        }
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        pl.stats.queued = (int32_t)std::min<size_t>(pl.queue.size(), INT32_MAX);
    }
    if (pl.queue.empty()) return false;
    const int32_t k = pl.queue.front().k;
    for (auto it = pl.queue.begin(); it != pl.queue.end() && (int)pl.running.size() < kPlainGroup;) {
        if (it->k == k) {
            pl.h_seeds[pl.running.size()] = it->seed;
            pl.running.push_back(*it);
            it = pl.queue.erase(it);
        } else {
            ++it;
        }
    }
    const int m = (int)pl.running.size();
    pl.t_admit = mono_ns();
    KHOP_HIP(hipMemcpyAsync(pl.d_seeds, pl.h_seeds, (size_t)m * 4, hipMemcpyHostToDevice, pl.stream));
    KHOP_HIP(hipEventRecord(pl.ev_start, pl.stream));
    khop::plain_run(pl.g, pl.ctx, pl.d_seeds, m, k, pl.d_counts, nullptr, pl.stream);
    KHOP_HIP(hipEventRecord(pl.ev_stop, pl.stream));
    KHOP_HIP(hipMemcpyAsync(pl.h_counts, pl.d_counts, (size_t)m * 8, hipMemcpyDeviceToHost, pl.stream));
    KHOP_HIP(hipEventRecord(pl.ev_end, pl.stream));
    pl.inflight = true;
    return true;
}

void scheduler(khop_server *s) {
    try {
        bool device_set = false;
        while (true) {
            std::vector<BatchLane *> lanes;
            std::vector<PlainLane *> plains;
            std::deque<ServeRequest> arrived;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                if (s->stop) break;
                lanes = s->lanes;
                plains = s->plains;
                arrived.swap(s->incoming);
            }
            if (!lanes.empty() && !device_set) {
                KHOP_HIP(hipSetDevice(lanes[0]->g->device));
                device_set = true;
            }
            bool busy = false;
            // completed work first: it frees slots and sharpens the estimates the routing uses
            for (PlainLane *pl : plains) {
                if (!pl->inflight) continue;
                if (hipEventQuery(pl->ev_end) != hipSuccess) {
                    busy = true;
                    continue;
                }
                pl->inflight = false;
                complete_plain(s, *pl);
            }
            int64_t now = mono_ns();
            for (BatchLane *L : lanes) busy |= poll_lane(s, *L, now);
            const int route = s->route.load();
            for (const ServeRequest &r : arrived) {
                if (r.k == 0) {
                    finish(s, r, KHOP_OK, 0, now);
                    continue;
                }
                PlainLane &pl = *plains[r.graph_id];
                BatchLane &L = *lanes[khop::serve_lane_of(r.graph_id, r.k)];
                if (s->router.take(route, now, pl.floor_cost(r.k), pl.cost(r.k), pl.backlog_ms,
                                   khop::lane_latency_ms(L.plan, now))) {
                    ServeRequest q = r;
                    q.plain_ms = pl.cost(r.k);
                    pl.backlog_ms += q.plain_ms;
                    pl.queue.push_back(q);
                } else {
                    L.plan.queue.push_back(r);
                }
            }
            now = mono_ns();
            for (PlainLane *pl : plains) {
                if (pl->inflight) continue;
                busy |= plan_plain(s, *pl, now);
                busy |= !pl->queue.empty();
            }
            int64_t avail = s->budget - s->used;
            bool waiting = false;
            for (BatchLane *L : lanes) busy |= plan_batch_lane(s, *L, now, avail, waiting);
            s->used = s->budget - avail;
            s->waiting_mem = waiting;
            if (!busy) {
                std::unique_lock<std::mutex> lk(s->mu);
                if (!s->stop && s->incoming.empty()) s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
            } else {
                std::this_thread::sleep_for(std::chrono::microseconds(5));
            }
        }
    } catch (const khop::Error &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->thread_error = e.msg;
        s->stop = true;
        s->cv_done.notify_all();
    } catch (...) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->thread_error = "scheduler failed";
        s->stop = true;
        s->cv_done.notify_all();
    }
}

void free_plain_lane(PlainLane *pl) {
    if (!pl) return;
    if (pl->stream) (void)hipStreamSynchronize(pl->stream);
    if (pl->ctx) khop::plain_ctx_destroy(pl->ctx);
    if (pl->d_seeds) (void)hipFree(pl->d_seeds);
    if (pl->d_counts) (void)hipFree(pl->d_counts);
    if (pl->h_seeds) (void)hipHostFree(pl->h_seeds);
    if (pl->h_counts) (void)hipHostFree(pl->h_counts);
    if (pl->ev_start) (void)hipEventDestroy(pl->ev_start);
    if (pl->ev_stop) (void)hipEventDestroy(pl->ev_stop);
    if (pl->ev_end) (void)hipEventDestroy(pl->ev_end);
    if (pl->stream) (void)hipStreamDestroy(pl->stream);
    delete pl;
}

void free_batch_lane(BatchLane *L) {
    if (!L) return;
    for (RunRes &R : L->res) {
        if (R.stream) (void)hipStreamSynchronize(R.stream);
        if (R.ctx) khop::batch_ctx_destroy(R.ctx);
        if (R.d_seeds) (void)hipFree(R.d_seeds);
        if (R.d_counts) (void)hipFree(R.d_counts);
        if (R.h_seeds) (void)hipHostFree(R.h_seeds);
        if (R.h_counts) (void)hipHostFree(R.h_counts);
        if (R.done) (void)hipEventDestroy(R.done);
        if (R.stream) (void)hipStreamDestroy(R.stream);
    }
    delete L;
}

template <class F>
int sguard(F &&f) {
    try {
        f();
        return KHOP_OK;
    } catch (const khop::Error &e) {
        khop::set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        khop::set_last_error("host allocation failed");
        return KHOP_ENOMEM;
    } catch (...) {
        khop::set_last_error("internal error");
        return KHOP_EINTERNAL;
    }
}

}  // namespace

extern "C" {

int khop_server_create(int64_t mem_budget_bytes, int32_t max_batch_seeds, khop_server **out) {
    return sguard([&] {
        if (!out) khop::fail(KHOP_EINVAL, "out is NULL");
        if (mem_budget_bytes <= 0) khop::fail(KHOP_EINVAL, "mem_budget_bytes must be positive");
        if (max_batch_seeds < 64 || max_batch_seeds > 1024 || max_batch_seeds % 64)
            khop::fail(KHOP_EINVAL, "max_batch_seeds must be a multiple of 64 in [64, 1024]");
        auto *s = new khop_server();
        s->budget = mem_budget_bytes;
        s->max_words = max_batch_seeds / 64;
        s->th = std::thread(scheduler, s);
        *out = s;
    });
}

int khop_server_batch_bytes(const khop_graph *g, int32_t words, int64_t *bytes) {
    return sguard([&] {
        if (!g || !bytes) khop::fail(KHOP_EINVAL, "graph or bytes is NULL");
        if (words < 1 || words > 16) khop::fail(KHOP_EINVAL, "words must be in [1, 16]");
        *bytes = (int64_t)khop::batch_ctx_bytes(g->n, g->nnz, words);
    });
}

int khop_server_add_graph(khop_server *s, khop_graph *g, int32_t *graph_id) {
    return sguard([&] {
        if (!s || !g || !graph_id) khop::fail(KHOP_EINVAL, "server, graph or graph_id is NULL");
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) khop::fail(KHOP_EINTERNAL, "server stopped: " + s->thread_error);
        if (!s->lanes.empty() && s->lanes[0]->g->device != g->device)
            khop::fail(KHOP_EINVAL, "all graphs of a server must live on one device");
        KHOP_HIP(hipSetDevice(g->device));
        const int id = s->ngraphs;
        auto *pl = new PlainLane();
        pl->g = g;
        pl->graph_id = id;
        std::vector<BatchLane *> made;
        try {
            KHOP_HIP(hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking));
            // timing events without a system-scope fence, so recording them writes back no cache
            KHOP_HIP(hipEventCreateWithFlags(&pl->ev_start, hipEventDisableSystemFence));
            KHOP_HIP(hipEventCreateWithFlags(&pl->ev_stop, hipEventDisableSystemFence));
            KHOP_HIP(hipEventCreateWithFlags(&pl->ev_end, hipEventDisableTiming));
            if (hipMalloc(&pl->d_seeds, kPlainGroup * 4) != hipSuccess ||
                hipMalloc(&pl->d_counts, kPlainGroup * 8) != hipSuccess ||
                hipHostMalloc((void **)&pl->h_seeds, kPlainGroup * 4, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void **)&pl->h_counts, kPlainGroup * 8, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                khop::fail(KHOP_ENOMEM, "allocation for a single-query lane failed");
            }
            pl->ctx = khop::plain_ctx_create(g);
            const size_t cap = (size_t)64 * s->max_words;
            for (int l = 0; l < khop::kServeLanes; ++l) {
                auto *L = new BatchLane();
                made.push_back(L);
                L->g = g;
                L->graph_id = id;
                L->lane = l;
                for (RunRes &R : L->res) {
                    KHOP_HIP(hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking));
                    KHOP_HIP(hipEventCreateWithFlags(&R.done, hipEventDisableTiming));
                    if (hipMalloc(&R.d_seeds, cap * 4) != hipSuccess || hipMalloc(&R.d_counts, cap * 8) != hipSuccess ||
                        hipHostMalloc((void **)&R.h_seeds, cap * 4, hipHostMallocDefault) != hipSuccess ||
                        hipHostMalloc((void **)&R.h_counts, cap * 8, hipHostMallocDefault) != hipSuccess) {
                        (void)hipGetLastError();
                        khop::fail(KHOP_ENOMEM, "allocation for a batch lane failed");
                    }
                }
            }
        } catch (...) {
            free_plain_lane(pl);
            for (BatchLane *L : made) free_batch_lane(L);
            throw;
        }
        s->plains.push_back(pl);
        for (BatchLane *L : made) s->lanes.push_back(L);
        *graph_id = s->ngraphs++;
    });
}

int khop_server_submit(khop_server *s, int32_t graph_id, int32_t seed, int32_t k, int64_t deadline_ns,
                       uint64_t *ticket) {
    return sguard([&] {
        if (!s || !ticket) khop::fail(KHOP_EINVAL, "server or ticket is NULL");
        if (k < 0) khop::fail(KHOP_EINVAL, "k < 0");
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) khop::fail(KHOP_EINTERNAL, "server stopped: " + s->thread_error);
        if (graph_id < 0 || graph_id >= s->ngraphs) khop::fail(KHOP_EINVAL, "unknown graph_id");
        if (seed < 0 || (int64_t)seed >= s->plains[graph_id]->g->n) khop::fail(KHOP_EINVAL, "seed out of range");
        if (s->incoming.size() >= kMaxQueued) khop::fail(KHOP_EBUSY, "request queue full");
        ServeRequest r;
        r.ticket = s->next_ticket++;
        r.graph_id = graph_id;
        r.seed = seed;
        r.k = k;
        r.t_submit = mono_ns();
        r.deadline = deadline_ns;
        s->incoming.push_back(r);
        s->submitted += 1;
        *ticket = r.ticket;
        s->cv_work.notify_one();
    });
}

int khop_server_set_option(khop_server *s, int32_t option, int64_t value) {
    return sguard([&] {
        if (!s) khop::fail(KHOP_EINVAL, "server is NULL");
        if (option != KHOP_SERVER_ROUTE) khop::fail(KHOP_EINVAL, "unknown server option");
        if (value != KHOP_ROUTE_AUTO && value != KHOP_ROUTE_BATCH && value != KHOP_ROUTE_PLAIN)
            khop::fail(KHOP_EINVAL, "route must be KHOP_ROUTE_AUTO, KHOP_ROUTE_BATCH or KHOP_ROUTE_PLAIN");
        s->route.store((int)value);
    });
}

int khop_server_poll(khop_server *s, khop_result *out, int64_t max, int64_t *n_out) {
    return sguard([&] {
        if (!s || !n_out || (max > 0 && !out)) khop::fail(KHOP_EINVAL, "server, out or n_out is NULL");
        std::lock_guard<std::mutex> lk(s->mu);
        int64_t n = 0;
        while (n < max && !s->done.empty()) {
            out[n++] = s->done.front();
            s->done.pop_front();
        }
        *n_out = n;
    });
}

int khop_server_stats(khop_server *s, khop_server_stat *out, int32_t max, int32_t *n_out) {
    return sguard([&] {
        if (!s || !n_out || (max > 0 && !out)) khop::fail(KHOP_EINVAL, "server, out or n_out is NULL");
        std::lock_guard<std::mutex> lk(s->mu);
        int32_t n = 0;
        auto put = [&](int32_t gid, int32_t lane, const LaneStats &st) {
            if (n < max) {
                khop_server_stat &o = out[n];
                o.graph_id = gid;
                o.lane = lane;
                o.launches = st.launches;
                o.queries = st.queries;
                o.busy_ms = st.busy_ms;
                o.max_ms = st.max_ms;
                o.words = st.words;
                o.queued = st.queued;
            }
            ++n;
        };
        for (BatchLane *L : s->lanes) put(L->graph_id, L->lane == 0 ? KHOP_LANE_SHORT : KHOP_LANE_DEEP, L->stats);
        for (PlainLane *pl : s->plains) put(pl->graph_id, KHOP_LANE_SINGLE, pl->stats);
        *n_out = std::min(n, std::max(max, 0));
    });
}

int khop_server_drain(khop_server *s, int64_t timeout_ms) {
    return sguard([&] {
        if (!s) khop::fail(KHOP_EINVAL, "server is NULL");
        std::unique_lock<std::mutex> lk(s->mu);
        const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(std::max<int64_t>(timeout_ms, 0)),
                                            [&] { return s->completed >= s->submitted || s->stop; });
        if (s->stop && s->completed < s->submitted) khop::fail(KHOP_EINTERNAL, "server stopped: " + s->thread_error);
        if (!ok) khop::fail(KHOP_ETIMEDOUT, "requests still pending after the timeout");
    });
}

int khop_server_destroy(khop_server *s) {
    return sguard([&] {
        if (!s) return;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->cv_work.notify_all();
        }
        if (s->th.joinable()) s->th.join();
        for (BatchLane *L : s->lanes) free_batch_lane(L);
        for (PlainLane *pl : s->plains) free_plain_lane(pl);
        delete s;
    });
}

}  // extern "C"
