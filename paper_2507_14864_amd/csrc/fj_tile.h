// Wave-level edge iteration over a tile of up to 64 consecutive CSR rows.
//
// A wave owns 64 consecutive rows.  Their arcs are one contiguous CSR range,
// which the 64 lanes stream in order (coalesced col/weight reads) regardless
// of how the degrees are distributed; each lane finds the row of its arc by a
// binary search over the row offsets kept in LDS (a merge-path split of the
// tile).  Per-row sums come out of a segmented scan across the lanes, added in
// a fixed order, so the result is identical run to run.
#pragma once
#include <type_traits>

#include "fj_device.h"

namespace fj {

// largest j in [0, cnt) with pre[j] <= e (pre nondecreasing, pre[0] <= e)
__device__ __forceinline__ int tile_find(const int* pre, int cnt, int e) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// FP64 sum over row (row0 + lane) of f(k) for every CSR position k of that
// row; lanes >= nrows get 0.  nrows in [0, 64], uniform across the wave.
// f may also take (k, slot), slot being the arc's row minus row0.  NCH
// 64-arc chunks are loaded together per step.
// pre: LDS [65] ints, acc: LDS [64] doubles, both private to this wave.
template <int NCH = 4, typename F>
__device__ __forceinline__ double tile_row_sums(const int32_t* __restrict__ row_ptr, int64_t row0, int nrows,
                                                int* pre, double* acc, F f) {
    const int lane = lane_id();
    if (nrows <= 0) return 0.0;
    int rb = lane < nrows ? row_ptr[row0 + lane] : 0;
    const int base = __shfl(rb, 0, 64);
    const int total = row_ptr[row0 + nrows] - base;
    if (lane < nrows) pre[lane] = rb - base;
    acc[lane] = 0.0;
    wave_sync_lds();
    auto reduce_chunk = [&](int key, double v) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double y = __shfl_up(v, o, 64);
            int ky = __shfl_up(key, o, 64);
            if (lane >= o && ky == key) v += y;
        }
        int knext = __shfl_down(key, 1, 64);
        if ((lane == 63 || knext != key) && key < 64) acc[key] += v;
        wave_sync_lds();
    };
    // NCH 64-arc chunks per step: their loads are in flight together
    for (int e0 = 0; e0 < total; e0 += 64 * NCH) {
        int key[NCH];
        double v[NCH];
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int e = e0 + 64 * j + lane;
            key[j] = 64 + lane;
            v[j] = 0.0;
            if (e < total) {
                key[j] = tile_find(pre, nrows, e);
                if constexpr (std::is_invocable_v<F, int, int>) v[j] = f(base + e, key[j]);
                else v[j] = f(base + e);
            }
        }
#pragma unroll
        for (int j = 0; j < NCH; ++j)
            if (e0 + 64 * j < total) reduce_chunk(key[j], v[j]);
    }
    return lane < nrows ? acc[lane] : 0.0;
}

// FP64 sum of f(k) over the arcs [beg, end) of one row chunk: lane-strided,
// then a fixed butterfly, so identical run to run.  Result in every lane.
template <typename F>
__device__ __forceinline__ double chunk_sum(int beg, int end, F f) {
    double acc = 0.0;
    int k = beg + lane_id();
    for (; k + 192 < end; k += 256) {  // four loads in flight per lane
        double a0 = f(k), a1 = f(k + 64), a2 = f(k + 128), a3 = f(k + 192);
        acc += a0; acc += a1; acc += a2; acc += a3;
    }
    for (; k < end; k += 64) acc += f(k);
    return wave_sum(acc);
}

// FP64 sum of f(k) over arcs [beg, end) by a whole block, in a fixed order:
// each thread takes U arcs per step (all U loads in flight together, the
// last step predicated), then a fixed butterfly per wave and the waves in
// index order.  Every thread of the block must call it; the total is
// returned to all.
template <int U = 4, typename F>
__device__ __forceinline__ double block_arc_sum(int beg, int end, double* lds /*[blockDim/64]*/, F f) {
    double acc = 0.0;
    const int nt = blockDim.x;
    for (int k = beg + static_cast<int>(threadIdx.x); k < end; k += U * nt) {
        double a[U];
#pragma unroll
        for (int j = 0; j < U; ++j) a[j] = k + j * nt < end ? f(k + j * nt) : 0.0;
#pragma unroll
        for (int j = 0; j < U; ++j) acc += a[j];
    }
    acc = wave_sum(acc);
    const int w = wave_id(), nw = nt >> 6;
    __syncthreads();
    if (lane_id() == 0) lds[w] = acc;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += lds[i];
    __syncthreads();
    return t;
}

// Same split without per-row sums: calls g(k, row_slot) for every CSR position
// of the tile.  Used where each arc's contribution is independent.
template <typename G>
__device__ __forceinline__ void tile_for_each_arc(const int32_t* __restrict__ row_ptr, int64_t row0, int nrows,
                                                  int* pre, G g) {
    const int lane = lane_id();
    if (nrows <= 0) return;
    int rb = lane < nrows ? row_ptr[row0 + lane] : 0;
    const int base = __shfl(rb, 0, 64);
    const int total = row_ptr[row0 + nrows] - base;
    if (lane < nrows) pre[lane] = rb - base;
    wave_sync_lds();
    for (int e = lane; e < total; e += 64) g(base + e, tile_find(pre, nrows, e));
    wave_sync_lds();
}

}  // namespace fj
