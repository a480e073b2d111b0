// Scheduling rules of the k-hop server, host code with no HIP dependency so
// that they can be checked on any host.
//
// The paper serves concurrent queries from a pool of workers, one query per
// worker (Section II).  On the GPU the server keeps the graphs resident and,
// per graph, runs two kinds of lanes:
//   - batch lanes (one for queries with k <= 2, one for deeper ones), each
//     with kRunsPerLane run slots.  A free slot takes the requests waiting in
//     its lane (FIFO, up to 64 per word of its context) as one batched launch
//     sequence -- seeds as bit columns, one bitset product per hop -- while
//     the lane's other slot may still be running: arrivals join the next
//     launch as soon as a slot and memory free up, and consecutive launches
//     overlap on the device.  A slot holds a batch context (its bitsets) only
//     while it is used, sized by the memory budget left;
//   - a single-query lane, which answers queries one at a time through the
//     plain path while the device time they would need stays low.
// Requests past their deadline leave the queues with a timeout status.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <numeric>
#include <vector>

namespace khop {

struct ServeRequest {
    uint64_t ticket = 0;
    int32_t graph_id = 0, seed = 0, k = 0;
    int64_t t_submit = 0, deadline = 0;  // CLOCK_MONOTONIC ns; deadline 0 = none
    double plain_ms = 0;                 // single-query lane: the cost charged to its backlog
};

constexpr int kServeLanes = 2;        // batch lanes per graph
constexpr int32_t kServeShortK = 2;   // queries with k up to this take lane 0
constexpr int kRunsPerLane = 2;       // batched launches a lane may have in flight
// An idle slot keeps its context this long (allocating and freeing a context
// of gigabytes costs milliseconds and synchronises the device, so a slot
// that is idle between launches at light load keeps it), unless another lane
// waits for memory.
constexpr int64_t kIdleReleaseNs = 2'000'000'000;
constexpr int64_t kSweepNs = 1'000'000;         // queued requests are checked for deadlines this often

inline int serve_lane_of(int32_t graph_id, int32_t k) {
    return graph_id * kServeLanes + (k > kServeShortK ? 1 : 0);
}

inline bool expired(const ServeRequest &r, int64_t now) { return r.deadline > 0 && now > r.deadline; }

// The order in which the queries of one batched launch take bit slots: by k,
// largest first, except that one-hop queries go last (they take no bit; a
// launch answers them from their seeds' rows).  Stable, so equal keys keep
// their arrival order.
inline std::vector<int32_t> batch_order(const int32_t *ks, int64_t n) {
    std::vector<int32_t> order((size_t)n);
    std::iota(order.begin(), order.end(), 0);
    auto key = [&](int32_t i) { return ks[i] == 1 ? -1 : ks[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key(a) > key(b); });
    return order;
}

// The widest batch context, in 64-seed words (a power of two up to
// max_words), whose bytes fit in avail; 0 when not even one word fits.
template <class Bytes>
int words_for_budget(int64_t avail, int max_words, Bytes &&bytes_of) {
    if ((int64_t)bytes_of(1) > avail) return 0;
    int w = 1;
    while (w * 2 <= max_words && (int64_t)bytes_of(w * 2) <= avail) w *= 2;
    return w;
}

// Moves up to cap requests from the front of q into batch, in arrival order;
// requests past their deadline met on the way go to late instead.
inline void take_batch(std::deque<ServeRequest> &q, int64_t now, int cap, std::vector<ServeRequest> &batch,
                       std::vector<ServeRequest> &late) {
    while (!q.empty() && (int)batch.size() < cap) {
        if (expired(q.front(), now)) late.push_back(q.front());
        else batch.push_back(q.front());
        q.pop_front();
    }
}

// Removes every request past its deadline from q (any position) into late.
inline void sweep_expired(std::deque<ServeRequest> &q, int64_t now, std::vector<ServeRequest> &late) {
    for (auto it = q.begin(); it != q.end();) {
        if (expired(*it, now)) {
            late.push_back(*it);
            it = q.erase(it);
        } else {
            ++it;
        }
    }
}

// One batch lane's host-side state.
struct LanePlan {
    struct Run {
        int words = 0;       // width of the slot's batch context (0: none held)
        int64_t bytes = 0;   // its device bytes, charged to the budget
        bool busy = false;   // a launch is in flight
        std::vector<ServeRequest> reqs;  // the requests of that launch, in slot order
        int64_t t_launch = 0, t_free = 0;
    };
    std::deque<ServeRequest> queue;
    Run runs[kRunsPerLane];
    double batch_ms = 2.0;  // moving average of a launch's time, enqueue to completion
    int64_t last_sweep = 0;
};

// What the scheduler does with one lane in one pass.  Launches are made on
// free slots, those already holding a context first; a slot without one gets
// the widest that the budget left (avail, updated) allows, or none, which
// sets waiting.  Each launch takes up to 64 * words queued requests; while
// another launch of the lane is in flight, a slot launches only when at least
// 16 * words requests wait (its width, or max_words without a context).  Idle
// slots give their context back after kIdleReleaseNs, or at once when some
// lane waits for memory (others_waiting).  Requests still queued after the
// launches whose deadline has passed leave the queue, at most every
// kSweepNs while requests wait only for a slot (the queue may be long), and
// in every pass while they wait for memory.
struct LaneActions {
    struct Launch {
        int run;
        int alloc_words;  // > 0: allocate a context this wide first
        std::vector<ServeRequest> batch;
    };
    std::vector<Launch> launches;
    std::vector<int> releases;  // slots whose context is freed (before any launch)
    std::vector<ServeRequest> late;
    bool waiting = false;
};

template <class Bytes>
LaneActions plan_lane(LanePlan &L, int64_t now, int64_t &avail, int max_words, bool others_waiting,
                      Bytes &&bytes_of) {
    LaneActions a;
    for (int i = 0; i < kRunsPerLane; ++i) {
        LanePlan::Run &r = L.runs[i];
        if (r.busy || r.words == 0 || !L.queue.empty()) continue;
        if (others_waiting || now - r.t_free >= kIdleReleaseNs) {
            a.releases.push_back(i);
            avail += r.bytes;
            r.words = 0;
            r.bytes = 0;
        }
    }
    int order[kRunsPerLane];
    std::iota(order, order + kRunsPerLane, 0);
    std::stable_sort(order, order + kRunsPerLane, [&](int x, int y) {
        return (L.runs[x].words > 0) > (L.runs[y].words > 0);
    });
    int in_flight = 0;
    for (const auto &r : L.runs) in_flight += r.busy;
    for (int oi = 0; oi < kRunsPerLane && !L.queue.empty(); ++oi) {
        const int i = order[oi];
        LanePlan::Run &r = L.runs[i];
        if (r.busy) continue;
        // beside a running launch, a second one starts only for a backlog of
        // a quarter of its width: a launch's fixed cost (one pass over the
        // graph per hop) is paid once for every query it holds
        const int width = r.words ? r.words : std::max(1, max_words);
        if (in_flight > 0 && (int64_t)L.queue.size() < 16 * (int64_t)width) break;
        int alloc = 0;
        if (r.words == 0) {
            alloc = words_for_budget(avail, max_words, bytes_of);
            if (alloc == 0) {
                a.waiting = true;
                break;
            }
        }
        std::vector<ServeRequest> batch;
        take_batch(L.queue, now, 64 * (alloc ? alloc : r.words), batch, a.late);
        if (batch.empty()) break;  // only late requests were left
        if (alloc) {
            r.words = alloc;
            r.bytes = (int64_t)bytes_of(alloc);
            avail -= r.bytes;
        }
        r.busy = true;
        r.reqs = batch;
        r.t_launch = now;
        a.launches.push_back({i, alloc, std::move(batch)});
        ++in_flight;
    }
    if (!L.queue.empty() && (a.waiting || now - L.last_sweep >= kSweepNs)) {
        L.last_sweep = now;
        sweep_expired(L.queue, now, a.late);
    }
    return a;
}

// A launch on slot i has completed at time now.
inline void complete_run(LanePlan &L, int i, int64_t now) {
    LanePlan::Run &r = L.runs[i];
    L.batch_ms = 0.7 * L.batch_ms + 0.3 * (double)(now - r.t_launch) / 1e6;
    r.busy = false;
    r.reqs.clear();
    r.t_free = now;
}

// How long a request joining the lane now should wait for its count: the
// launch it joins starts when a slot is free, and takes about batch_ms.
inline double lane_latency_ms(const LanePlan &L, int64_t now) {
    double wait = 1e30;
    for (const auto &r : L.runs) {
        if (!r.busy) return L.batch_ms;
        wait = std::min(wait, std::max(0.0, L.batch_ms - (double)(now - r.t_launch) / 1e6));
    }
    return wait + L.batch_ms;
}

// Single-query demand: the device time the single-query lanes would need for
// the arrivals, as a fraction of wall time, as an exponentially decayed sum
// over kDemandNs.  Cheap queries (uncontended cost up to kCheapMs) take those
// lanes while their own demand stays below kCheapLoad; dearer ones only while
// the demand of all arrivals stays below the device (entered below
// kDemandLow, left above kDemandHigh).  Beyond that the batches are the
// cheaper way to answer.
struct Demand {
    static constexpr double kDemandNs = 5e6;
    double acc = 0;
    int64_t t = 0;
    double add(int64_t now, double ms) {
        acc = acc * std::exp(-(double)(now - t) / kDemandNs) + ms;
        t = now;
        return acc / (kDemandNs / 1e6);  // device ms per wall ms
    }
};

enum { ROUTE_AUTO = 0, ROUTE_BATCH = 1, ROUTE_PLAIN = 2 };

struct SingleRouter {
    static constexpr double kCheapMs = 0.05, kCheapLoad = 0.5, kDemandLow = 0.8, kDemandHigh = 1.0;
    // The single-query lane is for latency at light load: it never queues more
    // than this much of its measured per-query device time (its costs rise
    // when batches share the device, so a long queue there would wait longer
    // than the batches take).
    static constexpr double kMaxBacklogMs = 3.0;
    Demand all, cheap;
    bool plain_mode = true;  // the single-query lanes take queries that are not cheap
    // Whether the single-query lane answers a request: its uncontended cost
    // floor_ms, the lane's current per-query estimate cost_ms and backlog, and
    // the latency a batch lane would give it.  The lane must also be expected
    // to answer first, within kMaxBacklogMs.
    bool take(int route, int64_t now, double floor_ms, double cost_ms, double backlog_ms, double batch_ms) {
        if (route == ROUTE_BATCH) return false;
        if (route == ROUTE_PLAIN) return true;
        const double load = all.add(now, floor_ms);
        if (plain_mode && load > kDemandHigh) plain_mode = false;
        if (!plain_mode && load < kDemandLow) plain_mode = true;
        if (floor_ms <= kCheapMs) {
            if (cheap.add(now, floor_ms) > kCheapLoad) return false;
        } else if (!plain_mode) {
            return false;
        }
        return backlog_ms + cost_ms <= std::min(batch_ms, kMaxBacklogMs);
    }
};

}  // namespace khop
