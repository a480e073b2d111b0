// Autotuner (placeholder until the search is in place).
#include "khop_impl.h"

extern "C" int khop_autotune(khop_graph *g, int32_t seeds_per_launch) {
    (void)seeds_per_launch;
    if (!g) return KHOP_EINVAL;
    return KHOP_EINTERNAL;
}
