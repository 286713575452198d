// Graph ingest: validation, degrees, CSR(A^T), colouring of A + A^T and the
// colour-ordered relabelled copy of A.
//
// d_i = sum_j a_ij and L = D - A (Sec. 3.2).  A push at v hands residual to
// every u with a_uv > 0, which is column v of A (proof of Lemma 4), so directed
// graphs also get CSR(A^T).  Over-relaxed sweeps need an order in which
// simultaneously updated rows do not read each other; colour classes of the
// symmetrised pattern give such an order, and within a class the simultaneous
// row updates equal the sequential Gauss-Seidel updates of Thm. 8.
#include <algorithm>
#include <cstring>

#include "fj_device.h"
#include "fj_internal.h"

namespace fj {

// ------------------------------------------------------------------- scan
namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int block_excl_scan_int(int v, int* lds /*[kScanThreads/64]*/, int* total) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    int incl = wave_incl_scan(v);
    if (lane == 63) lds[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        int t = lds[i];
        if (i < w) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(const int32_t* in, int64_t n, int32_t* bsum) {
    __shared__ int lds[kScanThreads / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int tot;
    block_excl_scan_int(s, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_bsum(int32_t* bsum, int64_t nb) {
    __shared__ int lds[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        int64_t i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        const int lane = lane_id(), w = threadIdx.x >> 6;
        int incl = wave_incl_scan(v);
        if (lane == 63) lds[w] = incl;
        __syncthreads();
        int off = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            int t = lds[k];
            if (k < w) off += t;
            tot += t;
        }
        int c = carry;
        if (i < nb) bsum[i] = c + off + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* in, int32_t* out, int64_t n,
                                                             const int32_t* bsum) {
    __shared__ int lds[kScanThreads / 64];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int off = block_excl_scan_int(s, lds, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
}
}  // namespace

size_t scan_tmp_bytes(int64_t n) { return sizeof(int32_t) * static_cast<size_t>((n + kScanTile - 1) / kScanTile + 1); }

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* tmp, hipStream_t st) {
    if (n <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t* bsum = static_cast<int32_t*>(tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanThreads), 0, st, in, n, bsum);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, st, in, out, n, bsum);
}

// ------------------------------------------------------------- validation
namespace {
enum : int {
    kErrRowPtr = 1, kErrColRange = 2, kErrSelfLoop = 4, kErrUnsorted = 8, kErrWeight = 16, kErrAsym = 32
};

__global__ void k_validate_rows(int64_t n, int64_t nnz, const int32_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col, const float* __restrict__ w, int* err) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t b = row_ptr[i], e = row_ptr[i + 1];
    if (b < 0 || e < b || e > nnz) {
        atomicOr(err, kErrRowPtr);
        return;
    }
    int prev = -1, bad = 0;
    for (int64_t k = b; k < e; ++k) {
        int j = col[k];
        if (j < 0 || j >= n) { bad |= kErrColRange; break; }
        if (j == i) bad |= kErrSelfLoop;
        if (j <= prev) bad |= kErrUnsorted;
        prev = j;
        if (w) {
            float a = w[k];
            if (!(a > 0.0f) || !isfinite(a)) bad |= kErrWeight;
        }
    }
    if (bad) atomicOr(err, bad);
}

// Only run once k_validate_rows passed: every row range is inside [0, nnz] and
// every column is in range, so the binary search below stays in bounds.  A
// wave per row, its lanes striding over the row's arcs, so a hub's row is
// checked by 64 lanes instead of one thread.
__global__ void k_validate_symmetry(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    const float* __restrict__ w, int* err) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    for (int64_t k = row_ptr[i] + (threadIdx.x & 63); k < row_ptr[i + 1]; k += 64) {
        int j = col[k];
        int64_t lo = row_ptr[j], hi = row_ptr[j + 1] - 1, found = -1;
        while (lo <= hi) {
            int64_t mid = (lo + hi) >> 1;
            int c = col[mid];
            if (c == i) { found = mid; break; }
            if (c < i) lo = mid + 1; else hi = mid - 1;
        }
        if (found < 0 || (w && w[found] != w[k])) {
            atomicOr(err, kErrAsym);
            return;
        }
    }
}

// d_i = sum_j a_ij in FP64; 1 + d_i and its reciprocal
__global__ void k_degrees(int64_t n, const int32_t* __restrict__ row_ptr, const float* __restrict__ w,
                          double* opd, double* inv64, float* inv32, int* max_deg) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t b = row_ptr[i], e = row_ptr[i + 1];
    double d = 0.0;
    if (w) {
        for (int64_t k = b; k < e; ++k) d += static_cast<double>(w[k]);
    } else {
        d = static_cast<double>(e - b);
    }
    opd[i] = 1.0 + d;
    double inv = 1.0 / (1.0 + d);
    inv64[i] = inv;
    inv32[i] = static_cast<float>(inv);
    atomicMax(max_deg, static_cast<int>(e - b));
}

// ---------------------------------------------------------------- transpose
__global__ void k_count_cols(int64_t nnz, const int32_t* __restrict__ col, int32_t* cnt) {
    int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_transpose_scatter(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    const float* __restrict__ w, int32_t* cursor, int32_t* t_col, float* t_w) {
    // one wave per row: coalesced reads of the row, atomics spread over targets
    int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    for (int64_t k = row_ptr[i] + lane_id(); k < row_ptr[i + 1]; k += 64) {
        int j = col[k];
        int p = atomicAdd(&cursor[j], 1);
        t_col[p] = static_cast<int32_t>(i);
        if (t_w) t_w[p] = w ? w[k] : 1.0f;
    }
}

__global__ void k_max_row(int64_t n, const int32_t* __restrict__ row_ptr, int* mx) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(mx, row_ptr[i + 1] - row_ptr[i]);
}

// ----------------------------------------------------------------- colouring
// Jones-Plassmann with largest-degree-first priorities (ties broken by a hash
// of the label): a node takes the smallest colour unused by its higher-priority
// neighbours once all of them are coloured.  On a 10M-node power-law graph it
// gave fewer colours (62 against 67), and its colour order fewer sweeps (42
// against 45), than priorities by degree bucket floor(log2 d).  The result does
// not depend on thread timing: a node's colour is a function of its
// higher-priority neighbours' colours only.
__device__ __forceinline__ bool higher(uint64_t ku, int32_t u, uint64_t kv, int32_t v) {
    return ku > kv || (ku == kv && u > v);
}

// The colouring equals sequential first-fit in decreasing priority order; it is
// computed level by level.  Each node counts its higher-priority neighbours;
// a node whose count is zero is ready: its colour is the smallest one unused
// by those neighbours (all coloured already), after which it decrements the
// counts of its lower-priority neighbours, and those reaching zero form the
// next level.  One wave per node, scanning eight 64-arc chunks per step.
// Work is O(arcs) in total; the number of levels is the longest chain of
// decreasing priority (976 on the 10M-node graph), so most levels are small
// and are enqueued in batches without a host read of their sizes.

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}

__global__ void k_jp_init(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ t_row_ptr,
                          int directed, uint64_t* key, int32_t* colour) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t d = static_cast<uint32_t>(row_ptr[i + 1] - row_ptr[i]);
    if (directed) d += static_cast<uint32_t>(t_row_ptr[i + 1] - t_row_ptr[i]);
    key[i] = (static_cast<uint64_t>(d) << 32) | hash32(static_cast<uint32_t>(i) * 2654435761U + 17U);
    colour[i] = -1;
}

// number of higher-priority neighbours of v over one adjacency (wave-wide sum)
__device__ __forceinline__ int jp_count_higher(const int32_t* __restrict__ ptr, const int32_t* __restrict__ adj,
                                               int32_t v, uint64_t kv, const uint64_t* __restrict__ key) {
    int c = 0;
    for (int32_t k = ptr[v] + lane_id(); k < ptr[v + 1]; k += 64) {
        const int32_t u = adj[k];
        if (higher(key[u], u, kv, v)) ++c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    return c;
}

__global__ void k_jp_count(int64_t n, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ t_row_ptr, const int32_t* __restrict__ t_col, int directed,
                           const uint64_t* __restrict__ key, int32_t* wait, int32_t* ready, int* ready_count) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wave_id();
    if (w >= n) return;  // uniform across the wave
    const int32_t v = static_cast<int32_t>(w);
    const uint64_t kv = key[v];
    int c = jp_count_higher(row_ptr, col, v, kv, key);
    if (directed) c += jp_count_higher(t_row_ptr, t_col, v, kv, key);
    if (lane_id() == 0) {
        wait[v] = c;
        if (c == 0) ready[atomicAdd(ready_count, 1)] = v;
    }
}

// kJpChunks 64-arc chunks of v's adjacency per step: their loads (the
// neighbour, its key, its colour) are in flight together, so a hub's row
// costs a round trip per 512 arcs instead of per 64
constexpr int kJpChunks = 8;

// chunks first, first + stride, ... of v's adjacency (a wave: 0, 1; a block's
// wave w of W: w, W)
__device__ __forceinline__ uint64_t jp_used(const int32_t* __restrict__ ptr, const int32_t* __restrict__ adj,
                                            int32_t v, uint64_t kv, const uint64_t* __restrict__ key,
                                            const int32_t* __restrict__ colour, int base, int first = 0,
                                            int stride = 1) {
    uint64_t m = 0;
    const int32_t b = ptr[v], e = ptr[v + 1];
    for (int32_t k0 = b + 64 * first + lane_id(); k0 < e; k0 += 64 * stride * kJpChunks) {
        int32_t u[kJpChunks];
        int c[kJpChunks];
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j) {
            const int32_t k = k0 + 64 * stride * j;
            u[j] = k < e ? adj[k] : -1;
        }
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j)
            c[j] = u[j] >= 0 && higher(key[u[j]], u[j], kv, v) ? colour[u[j]] - base : -1;
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j)
            if (c[j] >= 0 && c[j] < 64) m |= 1ull << c[j];
    }
    return m;
}

// append, per lane, the values u[j] with take[j] set to list[*count ...]:
// one atomic per wave for all of them
template <int N>
__device__ __forceinline__ void wave_append_n(const bool* take, const int32_t* u, int* count, int32_t* list) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) c += take[j] ? 1 : 0;
    const int incl = wave_incl_scan(c);
    const int total = __shfl(incl, 63, 64);
    if (total == 0) return;
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(count, total);
    base = __shfl(base, 0, 64) + incl - c;
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (take[j]) list[base++] = u[j];
}

// the lower-priority neighbours of v lose one wait each; those reaching zero
// join the next level (kJpChunks chunks per step, their atomics in flight
// together)
__device__ __forceinline__ void jp_release(const int32_t* __restrict__ ptr, const int32_t* __restrict__ adj,
                                           int32_t v, uint64_t kv, const uint64_t* __restrict__ key, int32_t* wait,
                                           int32_t* next, int* next_count, int first = 0, int stride = 1) {
    const int32_t b = ptr[v], e = ptr[v + 1];
    // uniform trip count within the wave: the append needs every lane
    for (int32_t c0 = b + 64 * first; c0 < e; c0 += 64 * stride * kJpChunks) {
        int32_t u[kJpChunks];
        bool lower[kJpChunks], ready[kJpChunks];
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j) {
            const int32_t k = c0 + 64 * stride * j + lane_id();
            u[j] = k < e ? adj[k] : -1;
        }
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j) lower[j] = u[j] >= 0 && higher(kv, v, key[u[j]], u[j]);
#pragma unroll
        for (int j = 0; j < kJpChunks; ++j) ready[j] = lower[j] && atomicSub(&wait[u[j]], 1) == 1;
        wave_append_n<kJpChunks>(ready, u, next_count, next);
    }
}

// One priority level.  Its size is read on the device: counts[cur] holds it,
// the next level's nodes are appended to counts[(cur + 1) % 3], and
// counts[(cur + 2) % 3] (the size of the level before, no longer read) is
// cleared for the level after; so levels can be enqueued back to back
// without the host reading their sizes.  The waves stride over the level.
// counts[3] adds up the coloured nodes, counts[4] the non-empty levels.
// Nodes with kJpWideArcs or more arcs are left to k_jp_heavy (a block per
// node), listed in heavy[] with their count in hcount[par] (par: the level's
// parity; the other slot is cleared for the next level).  Nodes of one level
// are never adjacent, so the two kernels may colour them in either order.
constexpr int kJpWideArcs = 2048;

__global__ void k_jp_level(int* counts, int cur, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ t_row_ptr, const int32_t* __restrict__ t_col, int directed,
                           const uint64_t* __restrict__ key, int32_t* colour, int32_t* wait,
                           const int32_t* __restrict__ ready, int32_t* next, int32_t* heavy, int* hcount, int par) {
    const int count = __builtin_amdgcn_readfirstlane(counts[cur]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[(cur + 2) % 3] = 0;
        counts[3] += count;
        if (count > 0) counts[4] += 1;
        hcount[par ^ 1] = 0;
    }
    int* next_count = counts + (cur + 1) % 3;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wave_id(); w < count; w += nw) {
        const int32_t v = ready[w];
        int32_t deg = row_ptr[v + 1] - row_ptr[v];
        if (directed) deg += t_row_ptr[v + 1] - t_row_ptr[v];
        if (deg >= kJpWideArcs) {
            if (lane_id() == 0) heavy[atomicAdd(&hcount[par], 1)] = v;
            continue;
        }
        const uint64_t kv = key[v];
        for (int base = 0;; base += 64) {
            uint64_t m = jp_used(row_ptr, col, v, kv, key, colour, base);
            if (directed) m |= jp_used(t_row_ptr, t_col, v, kv, key, colour, base);
            m = wave_or(m);
            if (~m) {
                if (lane_id() == 0) colour[v] = base + __builtin_ctzll(~m);
                break;
            }
        }
        jp_release(row_ptr, col, v, kv, key, wait, next, next_count);
        if (directed) jp_release(t_row_ptr, t_col, v, kv, key, wait, next, next_count);
    }
}

// The wide nodes of the same level: a block of 16 waves per node, wave w
// taking chunks w, w + 16, ...; the used colours OR-ed across the block.
constexpr int kJpHeavyThreads = 1024;
__global__ __launch_bounds__(kJpHeavyThreads) void k_jp_heavy(int* counts, int cur, const int32_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const int32_t* __restrict__ t_row_ptr,
                                                              const int32_t* __restrict__ t_col, int directed,
                                                              const uint64_t* __restrict__ key, int32_t* colour,
                                                              int32_t* wait, int32_t* next,
                                                              const int32_t* __restrict__ heavy,
                                                              const int* hcount, int par) {
    __shared__ uint64_t s_or[kJpHeavyThreads / 64];
    constexpr int nwv = kJpHeavyThreads / 64;
    const int cnt = __builtin_amdgcn_readfirstlane(hcount[par]);
    const int wv = wave_id();
    int* next_count = counts + (cur + 1) % 3;
    for (int h = blockIdx.x; h < cnt; h += gridDim.x) {
        const int32_t v = heavy[h];
        const uint64_t kv = key[v];
        for (int base = 0;; base += 64) {
            uint64_t m = jp_used(row_ptr, col, v, kv, key, colour, base, wv, nwv);
            if (directed) m |= jp_used(t_row_ptr, t_col, v, kv, key, colour, base, wv, nwv);
            m = wave_or(m);
            if (lane_id() == 0) s_or[wv] = m;
            __syncthreads();
            uint64_t all = 0;
#pragma unroll
            for (int q = 0; q < nwv; ++q) all |= s_or[q];
            __syncthreads();  // s_or is written again by the next round
            if (~all) {
                if (threadIdx.x == 0) colour[v] = base + __builtin_ctzll(~all);
                break;
            }
        }
        jp_release(row_ptr, col, v, kv, key, wait, next, next_count, wv, nwv);
        if (directed) jp_release(t_row_ptr, t_col, v, kv, key, wait, next, next_count, wv, nwv);
    }
}

// max over rows i >= r0 of sum_{arcs j >= r0} a_ij / (1 + d_i), one wave per row
__global__ __launch_bounds__(256) void k_merge_coupling(int64_t r0, int64_t n, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col, const float* __restrict__ w,
                                                        const double* __restrict__ opd, unsigned long long* out) {
    const int64_t i = r0 + static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wave_id();
    if (i >= n) return;  // uniform across the wave
    double s = 0.0;
    for (int32_t k = row_ptr[i] + lane_id(); k < row_ptr[i + 1]; k += 64)
        if (col[k] >= r0) s += w ? static_cast<double>(w[k]) : 1.0;
    s = wave_sum(s);
    if (lane_id() == 0 && s > 0.0)
        atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(s / opd[i])));
}

__global__ void k_colour_count(int64_t n, const int32_t* __restrict__ colour, int* max_colour) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(max_colour, colour[i]);
}

// Stable counting sort of nodes by colour: per-chunk histograms, a scan in
// (colour, chunk) order, then an in-order scatter inside every chunk.
constexpr int kSortChunk = 1024;

__global__ __launch_bounds__(256) void k_colour_hist(int64_t n, const int32_t* __restrict__ colour, int K,
                                                     int32_t* hist, int64_t nchunks) {
    extern __shared__ int cnt[];
    for (int c = threadIdx.x; c < K; c += blockDim.x) cnt[c] = 0;
    __syncthreads();
    int64_t base = static_cast<int64_t>(blockIdx.x) * kSortChunk;
    for (int t = threadIdx.x; t < kSortChunk; t += blockDim.x)
        if (base + t < n) atomicAdd(&cnt[colour[base + t]], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < K; c += blockDim.x) hist[static_cast<int64_t>(c) * nchunks + blockIdx.x] = cnt[c];
}

// one wave per chunk, 64 nodes at a time in index order
__global__ __launch_bounds__(64) void k_colour_scatter(int64_t n, const int32_t* __restrict__ colour, int K,
                                                       const int32_t* __restrict__ off, int64_t nchunks,
                                                       int32_t* perm, int32_t* iperm) {
    extern __shared__ int run[];
    const int lane = lane_id();
    for (int c = lane; c < K; c += 64) run[c] = 0;
    wave_sync_lds();
    int64_t base = static_cast<int64_t>(blockIdx.x) * kSortChunk;
    for (int step = 0; step < kSortChunk / 64; ++step) {
        int64_t v = base + step * 64 + lane;
        bool valid = v < n;
        int c = valid ? colour[v] : -1;
        uint64_t todo = __ballot(valid);
        int rank = 0, grp = 0;
        bool leader = false;
        while (todo) {
            int l = __builtin_ctzll(todo);
            int lc = __shfl(c, l, 64);
            uint64_t m = __ballot(valid && c == lc);
            if (valid && c == lc) {
                rank = lanes_below(m);
                grp = __popcll(m);
                leader = (lane == l);
            }
            todo &= ~m;
        }
        int start = valid ? run[c] : 0;
        wave_sync_lds();
        if (valid) {
            int64_t pos = off[static_cast<int64_t>(c) * nchunks + blockIdx.x] + start + rank;
            perm[pos] = static_cast<int32_t>(v);
            iperm[v] = static_cast<int32_t>(pos);
            if (leader) run[c] = start + grp;
        }
        wave_sync_lds();
    }
}

__global__ void k_class_offsets(int K, const int32_t* __restrict__ off, int64_t nchunks, int64_t n, int64_t* class_off) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < K) class_off[c] = off[static_cast<int64_t>(c) * nchunks];
    if (c == K) class_off[K] = n;
}

__global__ void k_perm_rowlen(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ row_ptr,
                              int32_t* len) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        int32_t o = perm[i];
        len[i] = row_ptr[o + 1] - row_ptr[o];
    } else if (i == n) {
        len[n] = 0;
    }
}

// one wave per relabelled row
__global__ void k_perm_copy(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                            const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const float* __restrict__ w, const double* __restrict__ opd,
                            const double* __restrict__ inv64, const int32_t* __restrict__ prow_ptr, int32_t* pcol,
                            float* pw, double* popd, double* pinv64) {
    int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    int32_t o = perm[i];
    int32_t b = row_ptr[o], e = row_ptr[o + 1], pb = prow_ptr[i];
    for (int32_t k = b + lane_id(); k < e; k += 64) {
        pcol[pb + (k - b)] = iperm[col[k]];
        if (pw) pw[pb + (k - b)] = w[k];
    }
    if (lane_id() == 0 && popd) {
        popd[i] = opd[o];
        pinv64[i] = inv64[o];
    }
}

inline unsigned grid1d(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// ---------------------------------------------------------------- tile sets
__device__ __forceinline__ bool is_heavy(const int32_t* rp, int64_t i) { return rp[i + 1] - rp[i] > kArcBudget; }

__global__ void k_tile_mark(int64_t n, const int32_t* __restrict__ rp, int32_t* mark, int32_t* hm, int32_t* cm) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        mark[n] = 0; hm[n] = 0; cm[n] = 0;
        return;
    }
    bool hv = is_heavy(rp, i);
    bool start = (i % 64 == 0) || hv;
    if (i > 0) start = start || is_heavy(rp, i - 1) || (rp[i] / kArcBudget != rp[i - 1] / kArcBudget);
    mark[i] = start ? 1 : 0;
    hm[i] = hv ? 1 : 0;
    cm[i] = hv ? (rp[i + 1] - rp[i] + kArcBudget - 1) / kArcBudget : 0;
}

__global__ void k_seg_mark(const int64_t* __restrict__ seg, int nseg, int64_t n, int32_t* mark) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nseg && seg[k] < n) mark[seg[k]] = 1;
}

__global__ void k_tile_fill(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ mark,
                            const int32_t* __restrict__ tscan, const int32_t* __restrict__ hscan,
                            const int32_t* __restrict__ cscan, int32_t* tile_start, int32_t* tile_heavy,
                            int32_t* heavy_row, int32_t* heavy_chunk0, int32_t* chunk_heavy, int32_t* chunk_beg,
                            int32_t* chunk_end) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        tile_start[tscan[n]] = static_cast<int32_t>(n);
        heavy_chunk0[hscan[n]] = cscan[n];
        return;
    }
    bool hv = is_heavy(rp, i);
    if (mark[i]) {
        tile_start[tscan[i]] = static_cast<int32_t>(i);
        tile_heavy[tscan[i]] = hv ? hscan[i] : -1;
    }
    if (hv) {
        int32_t h = hscan[i], c0 = cscan[i];
        heavy_row[h] = static_cast<int32_t>(i);
        heavy_chunk0[h] = c0;
        int32_t nch = (rp[i + 1] - rp[i] + kArcBudget - 1) / kArcBudget;
        for (int32_t j = 0; j < nch; ++j) {
            chunk_heavy[c0 + j] = h;
            chunk_beg[c0 + j] = rp[i] + j * kArcBudget;
            chunk_end[c0 + j] = min(rp[i] + (j + 1) * kArcBudget, rp[i + 1]);
        }
    }
}

__global__ void k_seg_offsets(const int64_t* __restrict__ seg, int nseg, const int32_t* __restrict__ tscan,
                              const int32_t* __restrict__ hscan, const int32_t* __restrict__ cscan, int32_t* out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nseg) return;
    int64_t row = seg[k];
    out[3 * k + 0] = tscan[row];
    out[3 * k + 1] = hscan[row];
    out[3 * k + 2] = cscan[row];
}

struct TileTemps {
    int32_t* mark; int32_t* tscan; int32_t* hscan; int32_t* cscan; int64_t* seg; int32_t* segout; void* scan_tmp;
};

void carve_tileset(Carver& cv, TileSet& T, int64_t n, int64_t nnz) {
    int64_t hmax = nnz / kArcBudget + 1;
    T.d_seg_tile = cv.take<int64_t>(kMaxColours + 2);
    T.d_seg_heavy = cv.take<int64_t>(kMaxColours + 2);
    T.tile_start = cv.take<int32_t>(n + 1);
    T.tile_heavy = cv.take<int32_t>(n + 1);
    T.heavy_row = cv.take<int32_t>(hmax);
    T.heavy_chunk0 = cv.take<int32_t>(hmax + 1);
    T.chunk_heavy = cv.take<int32_t>(2 * hmax + 2);
    T.chunk_beg = cv.take<int32_t>(2 * hmax + 2);
    T.chunk_end = cv.take<int32_t>(2 * hmax + 2);
}

// segments: sorted row starts, segs.front() = 0, segs.back() = n
fj_status build_tiles(TileSet& T, int64_t n, const int32_t* rp, const std::vector<int64_t>& segs,
                      const TileTemps& tmp, hipStream_t st) {
    const int bs = 256;
    const int nseg = static_cast<int>(segs.size()) - 1;
    FJ_HIP(hipMemcpyAsync(tmp.seg, segs.data(), sizeof(int64_t) * segs.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_tile_mark, dim3(grid1d(n + 1, bs)), dim3(bs), 0, st, n, rp, tmp.mark, tmp.hscan, tmp.cscan);
    if (nseg > 0) hipLaunchKernelGGL(k_seg_mark, dim3(grid1d(nseg, bs)), dim3(bs), 0, st, tmp.seg, nseg, n, tmp.mark);
    exclusive_scan_i32(tmp.mark, tmp.tscan, n + 1, tmp.scan_tmp, st);
    exclusive_scan_i32(tmp.hscan, tmp.hscan, n + 1, tmp.scan_tmp, st);
    exclusive_scan_i32(tmp.cscan, tmp.cscan, n + 1, tmp.scan_tmp, st);
    hipLaunchKernelGGL(k_tile_fill, dim3(grid1d(n + 1, bs)), dim3(bs), 0, st, n, rp, tmp.mark, tmp.tscan, tmp.hscan,
                       tmp.cscan, T.tile_start, T.tile_heavy, T.heavy_row, T.heavy_chunk0, T.chunk_heavy, T.chunk_beg,
                       T.chunk_end);
    hipLaunchKernelGGL(k_seg_offsets, dim3(grid1d(nseg + 1, bs)), dim3(bs), 0, st, tmp.seg, nseg, tmp.tscan, tmp.hscan,
                       tmp.cscan, tmp.segout);
    std::vector<int32_t> h(3 * (nseg + 1));
    FJ_HIP(hipMemcpyAsync(h.data(), tmp.segout, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    T.seg_tile.resize(nseg + 1);
    T.seg_heavy.resize(nseg + 1);
    T.seg_chunk.resize(nseg + 1);
    for (int k = 0; k <= nseg; ++k) {
        T.seg_tile[k] = h[3 * k];
        T.seg_heavy[k] = h[3 * k + 1];
        T.seg_chunk[k] = h[3 * k + 2];
    }
    T.ntiles = T.seg_tile[nseg];
    T.nheavy = T.seg_heavy[nseg];
    T.nchunks = T.seg_chunk[nseg];
    FJ_HIP(hipMemcpyAsync(T.d_seg_tile, T.seg_tile.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, st));
    FJ_HIP(hipMemcpyAsync(T.d_seg_heavy, T.seg_heavy.data(), sizeof(int64_t) * (nseg + 1), hipMemcpyHostToDevice, st));
    FJ_HIP(hipStreamSynchronize(st));
    return FJ_OK;
}

struct GraphLayout {
    double* opd; double* inv64; float* inv32;
    int32_t* t_row_ptr; int32_t* t_col; float* t_w; int32_t* t_cursor;
    int32_t* colour; uint64_t* key; int32_t* cur1; int32_t* cur2; int32_t* perm; int32_t* iperm;
    int32_t* hist; int64_t* class_off; int32_t* prow_ptr; int32_t* pcol; float* pw; double* popd; double* pinv64;
    int32_t* qrow_ptr; int32_t* qcol; float* qw;
    int* flags; void* scan_tmp;
    TileSet ta, tt, tp;
    TileTemps tmp;
};

constexpr int kMaxJpRounds = 1 << 16;

GraphLayout carve_graph(Carver& cv, const fj_graph_desc* d, int32_t flags) {
    GraphLayout L{};
    const int64_t n = d->n, nnz = d->nnz;
    const bool weighted = d->w != nullptr;
    L.opd = cv.take<double>(n);
    L.inv64 = cv.take<double>(n);
    L.inv32 = cv.take<float>(n);
    if (d->directed) {
        L.t_row_ptr = cv.take<int32_t>(n + 1);
        L.t_col = cv.take<int32_t>(nnz);
        L.t_w = weighted ? cv.take<float>(nnz) : nullptr;
        L.t_cursor = cv.take<int32_t>(n + 1);
    }
    L.flags = cv.take<int>(64);
    int64_t scan_n = n + 1;
    if (flags & FJ_GRAPH_COLOUR) {
        int64_t nchunks = (n + kSortChunk - 1) / kSortChunk;
        L.colour = cv.take<int32_t>(n);
        L.key = cv.take<uint64_t>(n);
        L.cur1 = cv.take<int32_t>(n);
        L.cur2 = cv.take<int32_t>(n);
        L.perm = cv.take<int32_t>(n);
        L.iperm = cv.take<int32_t>(n);
        L.hist = cv.take<int32_t>(static_cast<size_t>(kMaxColours) * nchunks);
        L.class_off = cv.take<int64_t>(kMaxColours + 1);
        L.prow_ptr = cv.take<int32_t>(n + 1);
        L.pcol = cv.take<int32_t>(nnz);
        L.pw = weighted ? cv.take<float>(nnz) : nullptr;
        L.popd = cv.take<double>(n);
        L.pinv64 = cv.take<double>(n);
        if (d->directed && !(flags & kGraphNoBoundCsr)) {
            L.qrow_ptr = cv.take<int32_t>(n + 1);
            L.qcol = cv.take<int32_t>(nnz);
            L.qw = weighted ? cv.take<float>(nnz) : nullptr;
        }
        scan_n = std::max<int64_t>(scan_n, static_cast<int64_t>(kMaxColours) * nchunks);
    }
    L.scan_tmp = cv.take<char>(scan_tmp_bytes(scan_n));
    carve_tileset(cv, L.ta, n, nnz);
    if (d->directed) carve_tileset(cv, L.tt, n, nnz);
    if (flags & FJ_GRAPH_COLOUR) carve_tileset(cv, L.tp, n, nnz);
    L.tmp.mark = cv.take<int32_t>(n + 1);
    L.tmp.tscan = cv.take<int32_t>(n + 1);
    L.tmp.hscan = cv.take<int32_t>(n + 1);
    L.tmp.cscan = cv.take<int32_t>(n + 1);
    L.tmp.seg = cv.take<int64_t>(kMaxColours + 2);
    L.tmp.segout = cv.take<int32_t>(3 * (kMaxColours + 2));
    L.tmp.scan_tmp = L.scan_tmp;
    return L;
}

}  // namespace

size_t graph_ws_bytes(const fj_graph_desc* d, int32_t flags) {
    Carver cv(nullptr);
    carve_graph(cv, d, flags);
    return cv.bytes();
}

fj_status graph_build(fj_graph* g, const fj_graph_desc* d, int32_t flags, void* ws, size_t ws_bytes, hipStream_t st) {
    const int64_t n = d->n, nnz = d->nnz;
    Carver cv(ws);
    GraphLayout L = carve_graph(cv, d, flags);
    if (cv.bytes() > ws_bytes) {
        set_error("graph workspace too small: need " + std::to_string(cv.bytes()) + " bytes");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    g->n = n;
    g->nnz = nnz;
    g->directed = d->directed ? 1 : 0;
    g->weighted = d->w ? 1 : 0;
    g->row_ptr = d->row_ptr;
    g->col = d->col;
    g->w = d->w;

    int* err = L.flags;  // flags[0..63] scratch scalars
    FJ_HIP(hipMemsetAsync(L.flags, 0, sizeof(int) * 64, st));
    int32_t ends[2] = {0, 0};
    FJ_HIP(hipMemcpyAsync(&ends[0], d->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipMemcpyAsync(&ends[1], d->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] != nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const int bs = 256;
    if (n > 0) hipLaunchKernelGGL(k_validate_rows, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, nnz, d->row_ptr, d->col, d->w, err);
    int herr = 0;
    FJ_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (herr == 0 && !d->directed && n > 0) {
        hipLaunchKernelGGL(k_validate_symmetry, dim3(grid1d(n * 64, bs)), dim3(bs), 0, st, n, d->row_ptr, d->col, d->w,
                           err);
        FJ_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
    }
    if (herr) {
        std::string m = "invalid CSR:";
        if (herr & kErrRowPtr) m += " row_ptr not nondecreasing within [0,nnz];";
        if (herr & kErrColRange) m += " column index out of range;";
        if (herr & kErrSelfLoop) m += " self-loop;";
        if (herr & kErrUnsorted) m += " row not strictly increasing (duplicate or unsorted);";
        if (herr & kErrWeight) m += " weight not finite and > 0;";
        if (herr & kErrAsym) m += " undirected graph is not symmetric;";
        set_error(m);
        return FJ_ERR_INVALID_ARGUMENT;
    }

    // degrees
    g->opd = L.opd;
    g->inv64 = L.inv64;
    g->inv32 = L.inv32;
    int* maxdeg = err + 1;
    int* maxin = err + 2;
    int* maxcol = err + 3;
    if (n > 0) hipLaunchKernelGGL(k_degrees, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, d->row_ptr, d->w, L.opd, L.inv64, L.inv32, maxdeg);

    // CSR(A^T)
    if (d->directed) {
        FJ_HIP(hipMemsetAsync(L.t_row_ptr, 0, sizeof(int32_t) * (n + 1), st));
        if (nnz > 0) hipLaunchKernelGGL(k_count_cols, dim3(grid1d(nnz, bs)), dim3(bs), 0, st, nnz, d->col, L.t_row_ptr);
        exclusive_scan_i32(L.t_row_ptr, L.t_row_ptr, n + 1, L.scan_tmp, st);
        FJ_HIP(hipMemcpyAsync(L.t_cursor, L.t_row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
        if (n > 0)
            hipLaunchKernelGGL(k_transpose_scatter, dim3(grid1d(n * 64, bs)), dim3(bs), 0, st, n, d->row_ptr, d->col,
                               d->w, L.t_cursor, L.t_col, L.t_w);
        if (n > 0) hipLaunchKernelGGL(k_max_row, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, L.t_row_ptr, maxin);
        g->t_row_ptr = L.t_row_ptr;
        g->t_col = L.t_col;
        g->t_w = L.t_w;
    } else {
        g->t_row_ptr = d->row_ptr;
        g->t_col = d->col;
        g->t_w = d->w;
    }
    int hdeg[2] = {0, 0};
    FJ_HIP(hipMemcpyAsync(hdeg, maxdeg, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    g->max_degree = hdeg[0];
    g->max_in_degree = d->directed ? hdeg[1] : hdeg[0];

    if (n > 0) {
        std::vector<int64_t> whole = {0, n};
        g->tiles_a = L.ta;
        fj_status rc = build_tiles(g->tiles_a, n, d->row_ptr, whole, L.tmp, st);
        if (rc) return rc;
        {  // can every heavy row of CSR(A) be combined in one launch?
            const TileSet& T = g->tiles_a;
            std::vector<int32_t> hc(T.nheavy + 1);
            FJ_HIP(hipMemcpyAsync(hc.data(), T.heavy_chunk0, sizeof(int32_t) * (T.nheavy + 1), hipMemcpyDeviceToHost,
                                  st));
            FJ_HIP(hipStreamSynchronize(st));
            g->a_packed = 1;
            for (int64_t h = 0; h < T.nheavy; ++h)
                if (hc[h + 1] - hc[h] > kMaxPackedChunks) g->a_packed = 0;
        }
        if (d->directed) {
            g->tiles_t = L.tt;
            rc = build_tiles(g->tiles_t, n, g->t_row_ptr, whole, L.tmp, st);
            if (rc) return rc;
        } else {
            g->tiles_t = g->tiles_a;
        }
    }

    if (!(flags & FJ_GRAPH_COLOUR) || n == 0) return FJ_OK;

    // Jones-Plassmann colouring, one priority level per launch (perm and iperm
    // hold the ready lists and cur1 the waiting counts until the relabelling
    // overwrites them)
    // counts[0..2]: level sizes in rotation (k_jp_level), [3] coloured nodes,
    // [4] levels, [5..6] wide nodes of the level by parity (their list in cur2)
    int* counts = err + 8;
    FJ_HIP(hipMemsetAsync(counts, 0, sizeof(int) * 7, st));
    hipLaunchKernelGGL(k_jp_init, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, d->row_ptr, g->t_row_ptr, g->directed,
                       L.key, L.colour);
    hipLaunchKernelGGL(k_jp_count, dim3(grid1d(n * 64, bs)), dim3(bs), 0, st, n, d->row_ptr, d->col, g->t_row_ptr,
                       g->t_col, g->directed, L.key, L.cur1, L.perm, counts);
    int level = 0;
    FJ_HIP(hipMemcpyAsync(&level, counts, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    // A level of at least kJpBigLevel nodes is launched alone with a wave per
    // node; smaller ones go kJpBatch at a time on a fixed grid, the host
    // reading the size only after each batch (a level past the last finds
    // size 0 and returns).
    constexpr int kJpBigLevel = 4096, kJpBatch = 32, kJpSmallBlocks = 512, kJpHeavyBlocks = 64;
    int64_t launched = 0;
    while (level > 0) {
        const int batch = level >= kJpBigLevel ? 1 : kJpBatch;
        if (launched + batch > kMaxJpRounds) {
            set_error("colouring did not finish within the round limit");
            return FJ_ERR_UNSUPPORTED;
        }
        for (int b = 0; b < batch; ++b, ++launched) {
            const unsigned grid = batch == 1 ? grid1d(static_cast<int64_t>(level) * 64, bs) : kJpSmallBlocks;
            int32_t* lin = launched % 2 == 0 ? L.perm : L.iperm;
            int32_t* lout = launched % 2 == 0 ? L.iperm : L.perm;
            const int cur = static_cast<int>(launched % 3), par = static_cast<int>(launched % 2);
            hipLaunchKernelGGL(k_jp_level, dim3(grid), dim3(bs), 0, st, counts, cur, d->row_ptr, d->col, g->t_row_ptr,
                               g->t_col, g->directed, L.key, L.colour, L.cur1, lin, lout, L.cur2, counts + 5, par);
            hipLaunchKernelGGL(k_jp_heavy, dim3(kJpHeavyBlocks), dim3(kJpHeavyThreads), 0, st, counts, cur,
                               d->row_ptr, d->col, g->t_row_ptr, g->t_col, g->directed, L.key, L.colour, L.cur1, lout,
                               L.cur2, counts + 5, par);
        }
        FJ_HIP(hipMemcpyAsync(&level, counts + launched % 3, sizeof(int), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
    }
    int tallies[2] = {0, 0};
    FJ_HIP(hipMemcpyAsync(tallies, counts + 3, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (tallies[0] != n) {
        set_error("colouring left nodes uncoloured");
        return FJ_ERR_UNSUPPORTED;
    }
    const int rounds = tallies[1];
    g->colour_rounds = rounds;
    hipLaunchKernelGGL(k_colour_count, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, L.colour, maxcol);
    int hmax = 0;
    FJ_HIP(hipMemcpyAsync(&hmax, maxcol, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    const int K = hmax + 1;
    if (K > kMaxColours) {
        set_error("graph needs " + std::to_string(K) + " colours; at most " + std::to_string(kMaxColours) +
                  " are supported");
        return FJ_ERR_UNSUPPORTED;
    }
    g->num_colours = K;
    g->colour = L.colour;

    // stable counting sort by colour -> perm (new -> old), iperm (old -> new)
    const int64_t nchunks = (n + kSortChunk - 1) / kSortChunk;
    hipLaunchKernelGGL(k_colour_hist, dim3(nchunks), dim3(256), sizeof(int) * K, st, n, L.colour, K, L.hist, nchunks);
    exclusive_scan_i32(L.hist, L.hist, static_cast<int64_t>(K) * nchunks, L.scan_tmp, st);
    hipLaunchKernelGGL(k_colour_scatter, dim3(nchunks), dim3(64), sizeof(int) * K, st, n, L.colour, K, L.hist,
                       nchunks, L.perm, L.iperm);
    hipLaunchKernelGGL(k_class_offsets, dim3(grid1d(K + 1, 256)), dim3(256), 0, st, K, L.hist, nchunks, n, L.class_off);
    g->class_off.assign(K + 1, 0);
    FJ_HIP(hipMemcpyAsync(g->class_off.data(), L.class_off, sizeof(int64_t) * (K + 1), hipMemcpyDeviceToHost, st));

    // relabelled CSR(A): row i is old row perm[i], columns mapped through iperm
    hipLaunchKernelGGL(k_perm_rowlen, dim3(grid1d(n + 1, bs)), dim3(bs), 0, st, n, L.perm, d->row_ptr, L.prow_ptr);
    exclusive_scan_i32(L.prow_ptr, L.prow_ptr, n + 1, L.scan_tmp, st);
    hipLaunchKernelGGL(k_perm_copy, dim3(grid1d(n * 64, bs)), dim3(bs), 0, st, n, L.perm, L.iperm, d->row_ptr, d->col,
                       d->w, L.opd, L.inv64, L.prow_ptr, L.pcol, L.pw, L.popd, L.pinv64);
    if (L.qrow_ptr) {
        // relabelled CSR(A^T): row i lists the rows of A that read node i (bound skipping)
        hipLaunchKernelGGL(k_perm_rowlen, dim3(grid1d(n + 1, bs)), dim3(bs), 0, st, n, L.perm, g->t_row_ptr,
                           L.qrow_ptr);
        exclusive_scan_i32(L.qrow_ptr, L.qrow_ptr, n + 1, L.scan_tmp, st);
        hipLaunchKernelGGL(k_perm_copy, dim3(grid1d(n * 64, bs)), dim3(bs), 0, st, n, L.perm, L.iperm, g->t_row_ptr,
                           g->t_col, g->t_w, nullptr, nullptr, L.qrow_ptr, L.qcol, L.qw, nullptr, nullptr);
    }
    FJ_HIP(hipStreamSynchronize(st));
    g->tiles_p = L.tp;
    {
        fj_status rc = build_tiles(g->tiles_p, n, L.prow_ptr, g->class_off, L.tmp, st);
        if (rc) return rc;
    }
    {  // classes whose heavy rows the one-launch sweep can combine
        const TileSet& T = g->tiles_p;
        std::vector<int32_t> hc(T.nheavy + 1), cb(T.nchunks), ce(T.nchunks);
        FJ_HIP(hipMemcpyAsync(hc.data(), T.heavy_chunk0, sizeof(int32_t) * (T.nheavy + 1), hipMemcpyDeviceToHost, st));
        if (T.nchunks > 0) {
            FJ_HIP(hipMemcpyAsync(cb.data(), T.chunk_beg, sizeof(int32_t) * T.nchunks, hipMemcpyDeviceToHost, st));
            FJ_HIP(hipMemcpyAsync(ce.data(), T.chunk_end, sizeof(int32_t) * T.nchunks, hipMemcpyDeviceToHost, st));
        }
        FJ_HIP(hipStreamSynchronize(st));
        g->heavy_arcs_p = 0;
        for (int64_t c = 0; c < T.nchunks; ++c) g->heavy_arcs_p += ce[c] - cb[c];
        g->class_packed.assign(K, 1);
        for (int k = 0; k < K; ++k)
            for (int64_t h = T.seg_heavy[k]; h < T.seg_heavy[k + 1]; ++h)
                if (hc[h + 1] - hc[h] > kMaxPackedChunks) g->class_packed[k] = 0;
    }
    // Tail merge analysis: the trailing small classes and, for every start T,
    // the largest coupling of a row to the rows of classes >= T
    g->merge_min = K;
    g->merge_coupling.assign(K + 1, 0.0);
    if (!g->directed && K >= 3) {
        std::vector<int32_t> bnd(K + 1);
        for (int k = 0; k <= K; ++k)
            FJ_HIP(hipMemcpyAsync(&bnd[k], L.prow_ptr + g->class_off[k], sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
        int T = K;
        while (T > 1 && g->class_packed[T - 1] &&
               static_cast<double>(bnd[T] - bnd[T - 1]) < kMergeArcFraction * static_cast<double>(nnz))
            --T;
        if (K - T >= 2) {
            unsigned long long* mc = reinterpret_cast<unsigned long long*>(L.tmp.seg);
            FJ_HIP(hipMemsetAsync(mc, 0, sizeof(unsigned long long) * (K + 1), st));
            for (int t = T; t < K; ++t) {
                const int64_t r0 = g->class_off[t];
                hipLaunchKernelGGL(k_merge_coupling, dim3(grid1d((n - r0) * 64, bs)), dim3(bs), 0, st, r0, n,
                                   L.prow_ptr, L.pcol, L.pw, L.popd, mc + t);
            }
            std::vector<unsigned long long> hm(K + 1);
            FJ_HIP(hipMemcpyAsync(hm.data(), mc, sizeof(unsigned long long) * (K + 1), hipMemcpyDeviceToHost, st));
            FJ_HIP(hipStreamSynchronize(st));
            for (int t = T; t < K; ++t) {
                double v;
                std::memcpy(&v, &hm[t], sizeof(double));
                g->merge_coupling[t] = v;
            }
            g->merge_min = T;
        }
    }
    g->perm = L.perm;
    g->iperm = L.iperm;
    g->prow_ptr = L.prow_ptr;
    g->pcol = L.pcol;
    g->pw = L.pw;
    g->qrow_ptr = L.qrow_ptr;
    g->qcol = L.qcol;
    g->qw = L.qw;
    g->popd = L.popd;
    g->pinv64 = L.pinv64;
    return FJ_OK;
}

}  // namespace fj
