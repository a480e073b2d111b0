// Drives the server's scheduling rules (serve_policy.h) on the host with a
// simulated clock and prints every decision as one JSON object per line, for
// tests/test_server_policy_cpu.py to check.
//
// Usage: serve_policy_sim SEED BUDGET MAX_WORDS LANES ARRIVALS
//        serve_policy_sim order K...   (prints batch_order of the ks)
//        serve_policy_sim route ROUTE GAP_NS FLOOR_MS COST_MS BATCH_MS N   (single-query routing)
//   Requests arrive at random times (seeded xorshift), each for a random lane
//   with a random k and, for one in five, a deadline.  A context of w words
//   costs 1000 + 300 * w bytes.  A launch of b requests completes
//   50 + 3 * b time units after it starts.  Each pass of the loop completes
//   due launches, then plans every lane, in the order the server does.  A
//   run whose queues never drain (a budget below one context) stops at time
//   10^6 and says so in its last line.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "serve_policy.h"

using namespace khop;

static uint64_t rng_state = 1;
static uint64_t next_u64() {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

int main(int argc, char **argv) {
    if (argc >= 2 && std::string(argv[1]) == "order") {
        // serve_policy_sim order K... : the slot order batch_order gives those ks
        std::vector<int32_t> ks;
        for (int i = 2; i < argc; ++i) ks.push_back(std::atoi(argv[i]));
        const std::vector<int32_t> o = batch_order(ks.data(), (int64_t)ks.size());
        for (size_t i = 0; i < o.size(); ++i) std::printf("%s%d", i ? " " : "", o[i]);
        std::printf("\n");
        return 0;
    }
    if (argc >= 2 && std::string(argv[1]) == "route") {
        // serve_policy_sim route ROUTE GAP_NS FLOOR_MS COST_MS BATCH_MS N : N arrivals GAP_NS apart; the
        // single-query lane serves its backlog at one device ms per wall ms.  One line per arrival:
        // taken (0/1) and the backlog after it.
        const int route = std::atoi(argv[2]);
        const int64_t gap = std::atoll(argv[3]);
        const double floor_ms = std::atof(argv[4]), cost_ms = std::atof(argv[5]), batch_ms = std::atof(argv[6]);
        const int n = std::atoi(argv[7]);
        SingleRouter router;
        double backlog = 0;
        int64_t now = 1;
        for (int i = 0; i < n; ++i, now += gap) {
            backlog = std::max(0.0, backlog - (double)gap / 1e6);
            const bool take = router.take(route, now, floor_ms, cost_ms, backlog, batch_ms);
            if (take) backlog += cost_ms;
            std::printf("%d %.6f\n", take ? 1 : 0, backlog);
        }
        return 0;
    }
    if (argc < 6) return 2;
    rng_state = 0x9e3779b97f4a7c15ull ^ std::strtoull(argv[1], nullptr, 10);
    const int64_t budget = std::atoll(argv[2]);
    const int max_words = std::atoi(argv[3]);
    const int nlanes = std::atoi(argv[4]);
    const int narr = std::atoi(argv[5]);
    auto bytes_of = [](int w) { return (int64_t)(1000 + 300 * w); };
    std::vector<LanePlan> lanes((size_t)nlanes);
    std::vector<std::vector<int64_t>> finish_at((size_t)nlanes, std::vector<int64_t>(kRunsPerLane, -1));
    int64_t now = 0, avail = budget;
    int arrived = 0;
    uint64_t ticket = 1;
    bool waiting = false;
    int64_t next_arrival = 0;
    const int64_t tmax = 1000000;  // a run that never drains (no memory) stops here
    while (now < tmax && (arrived < narr || [&] {
               for (auto &L : lanes) {
                   if (!L.queue.empty()) return true;
                   for (auto &r : L.runs)
                       if (r.busy) return true;
               }
               return false;
           }())) {
        // arrivals due by now
        while (arrived < narr && next_arrival <= now) {
            ServeRequest r;
            r.ticket = ticket++;
            const int lane = (int)(next_u64() % (uint64_t)nlanes);
            r.graph_id = lane;
            r.k = 1 + (int)(next_u64() % 7);
            r.t_submit = now;
            r.deadline = (next_u64() % 5 == 0) ? now + 1 + (int64_t)(next_u64() % 400) : 0;
            lanes[(size_t)lane].queue.push_back(r);
            std::printf("{\"ev\": \"arrive\", \"t\": %lld, \"lane\": %d, \"ticket\": %llu, \"deadline\": %lld}\n",
                        (long long)now, lane, (unsigned long long)r.ticket, (long long)r.deadline);
            ++arrived;
            next_arrival = now + (int64_t)(next_u64() % 12);
        }
        // completions
        for (int l = 0; l < nlanes; ++l)
            for (int i = 0; i < kRunsPerLane; ++i)
                if (lanes[(size_t)l].runs[i].busy && finish_at[(size_t)l][(size_t)i] <= now) {
                    std::printf("{\"ev\": \"done\", \"t\": %lld, \"lane\": %d, \"run\": %d}\n", (long long)now, l, i);
                    complete_run(lanes[(size_t)l], i, now);
                }
        // planning
        bool any_wait = false;
        for (int l = 0; l < nlanes; ++l) {
            LaneActions a = plan_lane(lanes[(size_t)l], now, avail, max_words, waiting, bytes_of);
            for (int i : a.releases)
                std::printf("{\"ev\": \"release\", \"t\": %lld, \"lane\": %d, \"run\": %d}\n", (long long)now, l, i);
            for (auto &r : a.late)
                std::printf("{\"ev\": \"late\", \"t\": %lld, \"lane\": %d, \"ticket\": %llu}\n", (long long)now, l,
                            (unsigned long long)r.ticket);
            for (auto &ln : a.launches) {
                const LanePlan::Run &r = lanes[(size_t)l].runs[ln.run];
                std::printf("{\"ev\": \"launch\", \"t\": %lld, \"lane\": %d, \"run\": %d, \"words\": %d, \"alloc\": %d, "
                            "\"bytes\": %lld, \"tickets\": [",
                            (long long)now, l, ln.run, r.words, ln.alloc_words, (long long)r.bytes);
                for (size_t j = 0; j < ln.batch.size(); ++j)
                    std::printf("%s%llu", j ? ", " : "", (unsigned long long)ln.batch[j].ticket);
                std::printf("]}\n");
                finish_at[(size_t)l][(size_t)ln.run] = now + 50 + 3 * (int64_t)ln.batch.size();
            }
            any_wait |= a.waiting;
        }
        waiting = any_wait;
        std::printf("{\"ev\": \"pass\", \"t\": %lld, \"avail\": %lld, \"waiting\": %d}\n", (long long)now,
                    (long long)avail, waiting ? 1 : 0);
        now += 1 + (int64_t)(next_u64() % 7);
    }
    // idle long enough: every context is given back
    now += kIdleReleaseNs;
    for (int l = 0; l < nlanes; ++l) {
        LaneActions a = plan_lane(lanes[(size_t)l], now, avail, max_words, false, bytes_of);
        for (int i : a.releases)
            std::printf("{\"ev\": \"release\", \"t\": %lld, \"lane\": %d, \"run\": %d}\n", (long long)now, l, i);
    }
    std::printf("{\"ev\": \"end\", \"avail\": %lld, \"budget\": %lld, \"cut\": %d}\n", (long long)avail,
                (long long)budget, now - kIdleReleaseNs >= tmax ? 1 : 0);
    return 0;
}
