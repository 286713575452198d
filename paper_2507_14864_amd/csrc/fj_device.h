// Device helpers for 64-wide CDNA wavefronts (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fj {

__device__ __forceinline__ int lane_id() { return __lane_id(); }
// this wave's index in its block, in a scalar register: the compiler then
// treats everything indexed by it (a row, a tile, a chunk) as wave-uniform
// and loads it with scalar loads instead of 64 lanes of the same address
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// index of this lane among the set lanes of `mask` below it
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// keeps the compiler from moving LDS traffic across this point within a wave
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// inclusive prefix sum over the wave (Hillis-Steele)
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// fixed-order butterfly reductions: identical results run to run
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-level fixed-order reduction of a double (block of kBlock threads).
// Every thread must call it.  Returns the total in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds /*[NT/64]*/) {
    v = wave_sum(v);
    const int w = wave_id();
    if (lane_id() == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < NT / 64; ++i) t += lds[i];
    }
    __syncthreads();
    return t;
}

// hardware float/double atomics (device memory from hipMalloc is coarse-grained)
__device__ __forceinline__ void atomic_add_noret(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_noret(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ float atomic_exch(float* p, float v) { return atomicExch(p, v); }
__device__ __forceinline__ double atomic_exch(double* p, double v) {
    unsigned long long old = atomicExch(reinterpret_cast<unsigned long long*>(p),
                                        static_cast<unsigned long long>(__double_as_longlong(v)));
    return __longlong_as_double(static_cast<long long>(old));
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

}  // namespace fj
