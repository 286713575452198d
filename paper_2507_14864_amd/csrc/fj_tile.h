// Wave-level edge iteration over a tile of up to 64 consecutive CSR rows.
//
// A wave owns 64 consecutive rows.  Their arcs are one contiguous CSR range,
// which the 64 lanes stream in order (coalesced col/weight reads) regardless
// of how the degrees are distributed; each lane finds the row of its arc by a
// binary search over the row offsets kept in LDS (a merge-path split of the
// tile).  Per-row sums come out of a segmented scan across the lanes, added in
// a fixed order, so the result is identical run to run.
#pragma once
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
// pre: LDS [65] ints, acc: LDS [64] doubles, both private to this wave.
template <typename F>
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
    for (int e0 = 0; e0 < total; e0 += 64) {
        const int e = e0 + lane;
        int key = 64 + lane;
        double v = 0.0;
        if (e < total) {
            key = tile_find(pre, nrows, e);
            v = f(base + e);
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double y = __shfl_up(v, o, 64);
            int ky = __shfl_up(key, o, 64);
            if (lane >= o && ky == key) v += y;
        }
        int knext = __shfl_down(key, 1, 64);
        if ((lane == 63 || knext != key) && key < 64) acc[key] += v;
        wave_sync_lds();
    }
    return lane < nrows ? acc[lane] : 0.0;
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
