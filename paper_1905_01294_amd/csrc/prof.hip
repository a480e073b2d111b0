// Profiling helper: a short bounded busy-wait launched ahead of each profiled
// kernel, so that the start event, the kernel and the end event are already
// queued when the device reaches them and the event pair brackets the kernel
// alone rather than also the host's enqueue latency.
#include "khop_impl.h"

namespace khop {
namespace {

__global__ void prof_delay_kernel(uint64_t ticks) {
    // wall clock at 100 MHz; the iteration cap bounds the wait whatever the clock does
    const uint64_t t0 = wall_clock64();
    for (int i = 0; i < (1 << 22); ++i) {
        if (wall_clock64() - t0 >= ticks) break;
        __builtin_amdgcn_s_sleep(2);
    }
}

__global__ void prof_empty_kernel() {}

}  // namespace

void prof_empty(hipStream_t st) { hipLaunchKernelGGL(prof_empty_kernel, dim3(1), dim3(64), 0, st); }

void prof_delay(hipStream_t st) {
    // about 200 us: longer than the host needs to enqueue the events and the kernel
    hipLaunchKernelGGL(prof_delay_kernel, dim3(1), dim3(64), 0, st, (uint64_t)20000);
}

}  // namespace khop
