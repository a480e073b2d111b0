// Wavefront-level helpers for gfx950 (64 lanes per wave).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace khop {
namespace dev {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// Number of set bits of m strictly below this lane.
__device__ __forceinline__ int mask_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= (uint64_t)__shfl_xor((long long)v, off, kWave);
    return v;
}

// Exclusive prefix sum over the wave's lanes.
__device__ __forceinline__ int64_t wave_exclusive_sum(int64_t v) {
    const int lane = lane_id();
    int64_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int64_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x - v;
}

// Column indices x .. x+3 in one 16-byte load (4-byte aligned).  The graph's
// column arrays carry four zero entries past their last index (kColidxPad),
// so that x may be any index below the array's length.
typedef int32_t i32x4_u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ i32x4_u load4(const int32_t *__restrict__ p, int64_t x) {
    return *(const i32x4_u *)(p + x);
}

__device__ __forceinline__ bool test_bit(const uint64_t *__restrict__ bm, int32_t v) {
    return (bm[(uint32_t)v >> 6] >> ((uint32_t)v & 63u)) & 1ull;
}

// Profiling counters of one launch: 4 fields x 64 lanes; each block adds to the
// lane of its index mod 64 so that no single address serialises the atomics.
constexpr int kUnitLanes = 64;
__device__ __forceinline__ void unit_add(int64_t *units, int field, int64_t v) {
    if (units && v)
        atomicAdd((unsigned long long *)&units[field * kUnitLanes + (blockIdx.x & (kUnitLanes - 1))],
                  (unsigned long long)v);
}

}  // namespace dev
}  // namespace khop
