// Prints the plain path's pipeline schedule (plain_plan.h) for the (k, m)
// pairs given on the command line, one JSON object per line: every step as
// [last, h1, marks, fin, setup], then the close launch.
#include <cstdio>
#include <cstdlib>

#include "plain_plan.h"

static void row(const khop::PlainStep &s) {
    std::printf("[%lld, %lld, %lld, %lld, %lld]", (long long)s.last, (long long)s.h1, (long long)s.marks,
                (long long)s.fin, (long long)s.setup);
}

int main(int argc, char **argv) {
    for (int i = 1; i + 1 < argc; i += 2) {
        const int k = std::atoi(argv[i]);
        const long long m = std::atoll(argv[i + 1]);
        std::printf("{\"k\": %d, \"m\": %lld, \"steps\": [", k, m);
        const long long n = khop::plain_plan_steps(k, m);
        for (long long j = 0; j < n; ++j) {
            if (j) std::printf(", ");
            row(khop::plain_plan_step(k, m, j));
        }
        std::printf("], \"close\": ");
        row(khop::plain_plan_close(m));
        std::printf("}\n");
    }
    return 0;
}
