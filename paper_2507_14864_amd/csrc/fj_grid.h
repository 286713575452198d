// Grid-wide barrier for kernels launched cooperatively (every block resident).
//
// A monotone arrival counter: barrier number b waits until the counter reaches
// gridDim.x * (b + 1), so the counter never needs resetting inside a launch
// (the host zeroes it before the launch).  Thread 0 of each block publishes
// the block's writes with an agent-scope release on its arrival and takes an
// agent-scope acquire after the wait; on gfx950 these are the L2 write-back
// and invalidate that make stores from other XCDs visible.  The wait is bounded
// by wall-clock time: if it expires (which cannot happen when all blocks are
// resident) the abort flag is raised and every block returns, so the kernel
// always drains.
#pragma once
#include "fj_device.h"

namespace fj {

// ~4 s at the 100 MHz constant clock read by wall_clock64()
constexpr long long kBarrierTimeoutTicks = 400000000LL;

struct GridSync {
    unsigned* counter;  // zeroed by the host before the launch
    int* abort;         // zeroed by the host before the launch
};

// Returns false if the barrier was aborted (the caller must return).
__device__ __forceinline__ bool grid_barrier(const GridSync& gs, unsigned& epoch) {
    __shared__ int s_ok;
    ++epoch;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = gridDim.x * epoch;
        __hip_atomic_fetch_add(gs.counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const long long t0 = wall_clock64();
        int ok = 1;
        while (__hip_atomic_load(gs.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(gs.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
            if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
                __hip_atomic_store(gs.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace fj
