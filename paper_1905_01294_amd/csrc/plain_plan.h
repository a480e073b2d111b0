// The schedule of the plain path's query pipeline: which query each piece of
// a step launch works on.  Host code with no HIP dependency, so that the
// schedule's invariants can be checked on any host.
//
// A run of m queries of k hops is: an init launch (query 0 set up), the
// steps 0..plain_plan_steps(k, m)-1, a close launch and a final launch.  Step
// j runs hop 1 of query j beside the last hop of query j-1 (k >= 2), and
// hops 2..k-1 of query j follow it in launches of their own.  A query's
// byte marks are counted by the launch after the one that ran its last hop,
// and its count is written by the launch after that.  Query q runs on bitmap
// state q % kPlanStates, control slot q % kPlanSlots and queue set
// q % kPlanQueueSets.
#pragma once

#include <cstdint>

namespace khop {

constexpr int kPlanStates = 3;
constexpr int kPlanSlots = 5;  // so that the count written and the query set up in a step never share one
constexpr int kPlanQueueSets = 2;

// The pieces of one launch; -1 where a piece is absent.
struct PlainStep {
    int64_t last;   // the query whose last hop (hop k >= 2) runs
    int64_t h1;     // the query whose hop 1 runs
    int64_t marks;  // the query whose byte marks are counted
    int64_t fin;    // the query whose count is written
    int64_t setup;  // the query set up: its control record written, its state reset (after the marks count)
};

inline int64_t plain_plan_steps(int32_t k, int64_t m) { return m <= 0 ? 0 : (k >= 2 ? m + 1 : m); }

// Step j, 0 <= j < plain_plan_steps(k, m).
inline PlainStep plain_plan_step(int32_t k, int64_t m, int64_t j) {
    PlainStep s;
    s.h1 = j < m ? j : -1;
    s.last = (k >= 2 && j >= 1) ? j - 1 : -1;
    const int64_t qm = k >= 2 ? j - 2 : j - 1;  // its last hop ran in the step before
    s.marks = qm >= 0 ? qm : -1;
    s.fin = qm >= 1 ? qm - 1 : -1;
    s.setup = j + 1 < m ? j + 1 : -1;
    return s;
}

// The close launch after the last step: the last query's marks and the
// count of the one before it.  (The final launch writes query m-1's count; a
// run of k = 1, which leaves no marks, has no close launch, and its final
// launch writes both counts.)
inline PlainStep plain_plan_close(int64_t m) {
    return PlainStep{-1, -1, m - 1, m >= 2 ? m - 2 : -1, -1};
}

}  // namespace khop
