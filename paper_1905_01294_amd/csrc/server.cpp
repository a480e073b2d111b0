// Continuous-batching server for k-hop queries.
//
// The paper serves many concurrent queries from a worker pool, one query per
// worker, arguing that throughput under concurrency matters more than the
// latency of one query on all cores (Section II).  Here the GPU analog: every
// resident graph has one running batched traversal whose 64*W seed-bit slots
// are refilled as queries finish.  A scheduler thread, per graph:
//   - when the graph's previous iteration has completed on its stream, turns
//     the counts it harvested into results;
//   - harvests slots whose query reached its k (bit-column popcount, bits
//     cleared), admits queued queries (FIFO) into free slots, and enqueues one
//     hop for every running slot -- new seeds go top-down from their seed,
//     running ones bottom-up in the shared bitset product;
//   - allocates a graph's batch only while it has work, sized by what the
//     memory budget still allows (3 bitsets of n words per 64 slots), so
//     queries wait rather than fail when memory is short.
// Each graph has two such batches ("lanes"), one for queries with k <= 2 and
// one for deeper ones, each on its own HIP stream: a short query never waits
// behind the hops of long ones, and lanes and graphs overlap on the device.
// Each graph also has a single-query lane on a third stream, which runs
// queries one after another through the plain path (the paper's one query
// per worker), in groups of one k.  A single query costs more device time
// than its share of a batch, the more so the deeper it goes, so the
// single-query lanes take arrivals only while the device time they would need
// stays low (decayed sums of the arrivals' uncontended costs: one for cheap
// queries, one for all, with hysteresis), and then only while the lane is
// expected to answer first (its backlog plus the query's cost, against k + 1
// measured iterations of the batch lane: k hops and the harvest).  So at low
// load every query gets the single-query latency; as load grows the deep ones
// and then the rest move into the batches, for their throughput.
#include <time.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>

#include "khop_impl.h"

namespace {

int64_t mono_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

struct Request {
    uint64_t ticket;
    int32_t graph_id, seed, k;
    int64_t t_submit, deadline;
    double plain_ms = 0;  // single-query lane: the cost charged to its backlog
};

struct Slot {
    bool used = false;
    int level = 0;
    Request req{};
    int64_t t_admit = 0;
};

struct GraphServe {
    khop_graph *g = nullptr;
    int id = 0;
    int lane = 0;  // 0: queries with k <= kShortK
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int64_t t_launch = 0;
    double it_ms = 0.5;  // moving average of one iteration's time, enqueue to completion
    khop::ServeCtx *ctx = nullptr;
    size_t ctx_bytes = 0;
    std::deque<Request> queue;
    std::vector<Slot> slots;
    bool inflight = false;
    std::vector<std::pair<int, Slot>> harvesting;  // slots whose counts the in-flight iteration produces
};

constexpr size_t kMaxQueued = 1 << 22;
constexpr int kLanes = 2;        // per graph
constexpr int32_t kShortK = 2;   // queries with k up to this go to lane 0
constexpr int kPlainGroup = 64;  // queries of one k per plain launch sequence
constexpr int kCostBuckets = 17; // per-k cost estimates; k >= 16 share the last
// Single-query demand: the device time the single-query lanes would need for
// the arrivals, as a fraction of wall time, averaged over kDemandNs.  Cheap
// queries (uncontended cost up to kCheapMs) take those lanes while their own
// demand stays below kCheapLoad; dearer ones only while the demand of all
// arrivals stays below the device (entered below kDemandLow, left above
// kDemandHigh).  Beyond that the batches are the cheaper way to answer.
constexpr double kDemandNs = 5e6;
constexpr double kCheapMs = 0.05;
constexpr double kCheapLoad = 0.5;
constexpr double kDemandLow = 0.8, kDemandHigh = 1.0;

// An exponentially decayed sum of device ms over wall time.
struct Demand {
    double acc = 0;
    int64_t t = 0;
    double add(int64_t now, double ms) {
        acc = acc * std::exp(-(double)(now - t) / kDemandNs) + ms;
        t = now;
        return acc / (kDemandNs / 1e6);  // device ms per wall ms
    }
};

int lane_of(int32_t graph_id, int32_t k) { return graph_id * kLanes + (k > kShortK ? 1 : 0); }

// The single-query lane of one graph.
struct PlainLane {
    khop_graph *g = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // timing only, around the launch sequence
    hipEvent_t ev_end = nullptr;                        // completion, after the counts' copy
    khop::PlainCtx *ctx = nullptr;
    int32_t *d_seeds = nullptr;  // kPlainGroup
    int64_t *d_counts = nullptr;
    int32_t *h_seeds = nullptr;  // pinned staging
    int64_t *h_counts = nullptr;
    std::deque<Request> queue;
    std::vector<Request> running;
    int64_t t_admit = 0;
    bool inflight = false;
    double cost_ms[kCostBuckets];   // moving average of one query's device time by k
    double floor_ms[kCostBuckets];  // the least per-query device time a group of that k took (uncontended)
    double backlog_ms = 0;          // expected device time of the queued and running queries
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
    int64_t used = 0;
    int max_words = 16;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<GraphServe *> graphs;  // kLanes lanes per graph, graph i's at [i * kLanes, (i + 1) * kLanes)
    std::vector<PlainLane *> plains;   // one per graph
    int ngraphs = 0;
    std::atomic<int> route{KHOP_ROUTE_AUTO};
    Demand demand_all, demand_cheap;  // arrivals' uncontended single-query cost
    bool plain_mode = true;           // the single-query lanes take queries that are not cheap
    std::deque<Request> incoming;
    std::deque<khop_result> done;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    int device = 0;
    std::thread th;
    std::string thread_error;
};

namespace {

void finish(khop_server *s, const Request &r, int status, int64_t count, int64_t t_admit,
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

// Results of the iteration that just completed on gs's stream.
void complete_iteration(khop_server *s, GraphServe &gs) {
    if (gs.harvesting.empty()) return;
    const int64_t *counts = khop::serve_ctx_counts(gs.ctx);
    for (auto &h : gs.harvesting) finish(s, h.second.req, KHOP_OK, counts[h.first] - 1, h.second.t_admit);
    gs.harvesting.clear();
}

bool ensure_ctx(khop_server *s, GraphServe &gs) {
    if (gs.ctx) return true;
    const int64_t avail = s->budget - s->used;
    if ((int64_t)khop::serve_ctx_bytes(gs.g->n, gs.g->nnz, 1) > avail) return false;
    int words = 1;
    while (words * 2 <= s->max_words && (int64_t)khop::serve_ctx_bytes(gs.g->n, gs.g->nnz, words * 2) <= avail)
        words *= 2;
    gs.ctx = khop::serve_ctx_create(gs.g, words);
    gs.ctx_bytes = khop::serve_ctx_bytes(gs.g->n, gs.g->nnz, words);
    s->used += (int64_t)gs.ctx_bytes;
    gs.slots.assign((size_t)64 * words, Slot{});
    return true;
}

void release_ctx(khop_server *s, GraphServe &gs) {
    if (!gs.ctx) return;
    KHOP_HIP(hipStreamSynchronize(gs.stream));
    khop::serve_ctx_destroy(gs.ctx);
    gs.ctx = nullptr;
    s->used -= (int64_t)gs.ctx_bytes;
    gs.ctx_bytes = 0;
    gs.slots.clear();
}

// Plans and enqueues one iteration; returns true if work was enqueued.
bool plan(khop_server *s, GraphServe &gs, int64_t now) {
    // queued requests past their deadline time out; k == 0 needs no traversal
    for (auto it = gs.queue.begin(); it != gs.queue.end();) {
        if (it->deadline > 0 && now > it->deadline) {
            finish(s, *it, KHOP_ETIMEDOUT, -1, 0);
            it = gs.queue.erase(it);
        } else if (it->k == 0) {
            finish(s, *it, KHOP_OK, 0, now);
            it = gs.queue.erase(it);
        } else {
            ++it;
        }
    }
    bool running = false;
    for (auto &sl : gs.slots) running |= sl.used;
    if (!running && gs.queue.empty()) {
        release_ctx(s, gs);  // idle: give the memory back
        return false;
    }
    if (!ensure_ctx(s, gs)) return false;  // waits for budget
    const int W = khop::serve_ctx_words(gs.ctx);
    std::vector<uint64_t> fin((size_t)W, 0), act((size_t)W, 0);
    std::vector<int32_t> new_slots, new_seeds;
    bool any_old = false;
    for (int j = 0; j < 64 * W; ++j) {
        Slot &sl = gs.slots[j];
        if (!sl.used) continue;
        if (sl.level >= sl.req.k) {
            fin[j >> 6] |= 1ull << (j & 63);
            gs.harvesting.push_back({j, sl});
            sl.used = false;
        } else {
            act[j >> 6] |= 1ull << (j & 63);
            any_old = true;
        }
    }
    for (int j = 0; j < 64 * W && !gs.queue.empty(); ++j) {
        Slot &sl = gs.slots[j];
        if (sl.used) continue;
        // a slot being harvested this iteration is cleared before the admission (stream order)
        sl.used = true;
        sl.level = 0;
        sl.req = gs.queue.front();
        sl.t_admit = now;
        gs.queue.pop_front();
        new_slots.push_back(j);
        new_seeds.push_back(sl.req.seed);
    }
    if (gs.harvesting.empty() && !any_old && new_slots.empty()) return false;
    // admission takes the lowest free slots, so the words holding live slots
    // are a prefix; the hop only works on it
    int wact = 1;
    for (int j = 0; j < 64 * W; ++j)
        if (gs.slots[j].used) wact = std::max(wact, (j >> 6) + 1);
    gs.t_launch = mono_ns();
    khop::serve_iteration(gs.ctx, fin.data(), act.data(), any_old, new_slots.data(), new_seeds.data(),
                          (int)new_slots.size(), wact, gs.stream);
    for (auto &sl : gs.slots)
        if (sl.used) sl.level += 1;
    KHOP_HIP(hipEventRecord(gs.ev, gs.stream));
    gs.inflight = true;
    return true;
}

// Which path answers request r first (the caller holds no lock; only the
// scheduler thread touches lanes).
bool route_plain(khop_server *s, const Request &r, int64_t now) {
    const int route = s->route.load();
    if (route == KHOP_ROUTE_BATCH) return false;
    if (route == KHOP_ROUTE_PLAIN) return true;
    const PlainLane &pl = *s->plains[r.graph_id];
    const double c = pl.floor_cost(r.k);
    const double load = s->demand_all.add(now, c);
    if (s->plain_mode && load > kDemandHigh) s->plain_mode = false;
    if (!s->plain_mode && load < kDemandLow) s->plain_mode = true;
    if (c <= kCheapMs) {
        if (s->demand_cheap.add(now, c) > kCheapLoad) return false;
    } else if (!s->plain_mode) {
        return false;
    }
    const GraphServe &gs = *s->graphs[lane_of(r.graph_id, r.k)];
    const double t_batch = (r.k + 1.5) * gs.it_ms;  // half an iteration in flight, k hops, the harvest
    return pl.backlog_ms + pl.cost(r.k) <= t_batch;
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
    pl.running.clear();
}

// Starts the next plain group: the oldest queued query and up to kPlainGroup - 1
// more of the same k, one launch sequence.  Returns true if work was enqueued.
bool plan_plain(khop_server *s, PlainLane &pl, int64_t now) {
    for (auto it = pl.queue.begin(); it != pl.queue.end();) {
        if (it->deadline > 0 && now > it->deadline) {
            pl.backlog_ms = std::max(0.0, pl.backlog_ms - it->plain_ms);
            finish(s, *it, KHOP_ETIMEDOUT, -1, 0, KHOP_PATH_SINGLE);
            it = pl.queue.erase(it);
        } else {
            ++it;
        }
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
            std::vector<GraphServe *> graphs;
            std::vector<PlainLane *> plains;
            std::deque<Request> arrived;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                if (s->stop) break;
                graphs = s->graphs;
                plains = s->plains;
                arrived.swap(s->incoming);
            }
            for (const Request &r : arrived) {
                if (r.k == 0) {
                    finish(s, r, KHOP_OK, 0, mono_ns());
                } else if (route_plain(s, r, mono_ns())) {
                    PlainLane &pl = *plains[r.graph_id];
                    Request q = r;
                    q.plain_ms = pl.cost(r.k);
                    pl.backlog_ms += q.plain_ms;
                    pl.queue.push_back(q);
                } else {
                    graphs[lane_of(r.graph_id, r.k)]->queue.push_back(r);
                }
            }
            const int64_t now = mono_ns();
            bool busy = false;
            if (!graphs.empty() && !device_set) {
                KHOP_HIP(hipSetDevice(graphs[0]->g->device));
                device_set = true;
            }
            for (PlainLane *pl : plains) {
                if (pl->inflight) {
                    if (hipEventQuery(pl->ev_end) != hipSuccess) {
                        busy = true;
                        continue;
                    }
                    pl->inflight = false;
                    complete_plain(s, *pl);
                }
                busy |= plan_plain(s, *pl, now);
                busy |= !pl->queue.empty();
            }
            for (GraphServe *gs : graphs) {
                if (gs->inflight) {
                    if (hipEventQuery(gs->ev) != hipSuccess) {
                        busy = true;
                        continue;
                    }
                    gs->inflight = false;
                    gs->it_ms = 0.7 * gs->it_ms + 0.3 * (double)(mono_ns() - gs->t_launch) / 1e6;
                    complete_iteration(s, *gs);
                }
                busy |= plan(s, *gs, now);
                busy |= !gs->queue.empty();
            }
            if (!busy) {
                std::unique_lock<std::mutex> lk(s->mu);
                if (!s->stop && s->incoming.empty())
                    s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
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

int khop_server_add_graph(khop_server *s, khop_graph *g, int32_t *graph_id) {
    return sguard([&] {
        if (!s || !g || !graph_id) khop::fail(KHOP_EINVAL, "server, graph or graph_id is NULL");
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) khop::fail(KHOP_EINTERNAL, "server stopped: " + s->thread_error);
        if (!s->graphs.empty() && s->graphs[0]->g->device != g->device)
            khop::fail(KHOP_EINVAL, "all graphs of a server must live on one device");
        KHOP_HIP(hipSetDevice(g->device));
        auto *pl = new PlainLane();
        pl->g = g;
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
        } catch (...) {
            free_plain_lane(pl);
            throw;
        }
        s->plains.push_back(pl);
        for (int l = 0; l < kLanes; ++l) {
            auto *gs = new GraphServe();
            gs->g = g;
            gs->id = s->ngraphs;
            gs->lane = l;
            KHOP_HIP(hipStreamCreateWithFlags(&gs->stream, hipStreamNonBlocking));
            KHOP_HIP(hipEventCreateWithFlags(&gs->ev, hipEventDisableTiming));
            s->graphs.push_back(gs);
        }
        s->device = g->device;
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
        if (seed < 0 || (int64_t)seed >= s->graphs[lane_of(graph_id, 0)]->g->n)
            khop::fail(KHOP_EINVAL, "seed out of range");
        if (s->incoming.size() >= kMaxQueued) khop::fail(KHOP_EBUSY, "request queue full");
        Request r{s->next_ticket++, graph_id, seed, k, mono_ns(), deadline_ns};
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
        for (GraphServe *gs : s->graphs) {
            if (gs->stream) (void)hipStreamSynchronize(gs->stream);
            if (gs->ctx) khop::serve_ctx_destroy(gs->ctx);
            if (gs->ev) (void)hipEventDestroy(gs->ev);
            if (gs->stream) (void)hipStreamDestroy(gs->stream);
            delete gs;
        }
        for (PlainLane *pl : s->plains) free_plain_lane(pl);
        delete s;
    });
}

}  // extern "C"
