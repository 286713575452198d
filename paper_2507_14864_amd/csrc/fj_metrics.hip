// Table 1 measures over z in FP64 with fixed-order reductions (bitwise
// reproducible): C = z^T z, I = sum (z - s)^2, P = sum (z - mean)^2 with the
// mean-centred vector of Sec. 3.4 (two passes, because the mean subtraction
// cancels), D = sum over edges of a_ij (z_i - z_j)^2 (undirected: each edge
// once, from its arc with j > i; directed: each arc once).
//
// The same passes accumulate what a-posteriori bounds on the measures need.
// If every |z_v - z*_v| <= b_v with b_v = kappa u_v, u_v = z_v + c (Lemma 7
// gives kappa = tau / (1 - tau) from the residual level tau, see
// fj_metrics_bounds), then expanding (x + e)^2 - x^2 = 2 x e + e^2 gives
//   |dC| <= kappa sum 2|z_v| u_v       + kappa^2 sum u_v^2
//   |dI| <= kappa sum 2|z_v - s_v| u_v + kappa^2 sum u_v^2
//   |dP| <= kappa sum 2|z_v - m| u_v   + kappa^2 sum u_v^2
//   |dD| <= kappa sum a_ij 2|z_i - z_j|(u_i + u_j) + kappa^2 sum a_ij (u_i + u_j)^2
// and the mean moves by at most kappa mean(u).  For P the centred values sum
// to zero, so the mean's move drops out of the first-order term and can only
// lower the second-order one.  The sums are formed once, before kappa is known.
#include <cmath>
#include <mutex>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_tile.h"

namespace fj {
namespace {

constexpr int kNodeItems = 8;
constexpr int kNodeTile = kBlock * kNodeItems;

inline unsigned nblocks_nodes(int64_t n) { return static_cast<unsigned>((n + kNodeTile - 1) / kNodeTile); }
inline unsigned nblocks_edges(const fj_graph* g) {
    return waves_to_blocks(g->tiles_a.nchunks + g->tiles_a.ntiles);
}

// device result slots
enum : int {
    kOutP = 0, kOutD, kOutI, kOutC, kOutMean,
    kOutUbar, kOutC1, kOutI1, kOutQ, kOutP1, kOutD1, kOutD2, kOutSlots
};
constexpr int kNodeStride = 7;

// pass 1 per block: sum z, z^2, (z - s)^2, u, 2|z| u, 2|z - s| u, u^2
__global__ __launch_bounds__(kBlock) void k_metrics_nodes(int64_t n, const double* __restrict__ s,
                                                          const double* __restrict__ z, double c, double* part) {
    __shared__ double lds[kWavesPerBlock];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kNodeTile + threadIdx.x;
    double acc[kNodeStride] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kNodeItems; ++k) {
        int64_t i = base + static_cast<int64_t>(k) * kBlock;
        if (i < n) {
            const double zi = z[i], d = zi - s[i], u = zi + c;
            acc[0] += zi;
            acc[1] += zi * zi;
            acc[2] += d * d;
            acc[3] += u;
            acc[4] += 2.0 * fabs(zi) * u;
            acc[5] += 2.0 * fabs(d) * u;
            acc[6] += u * u;
        }
    }
#pragma unroll
    for (int q = 0; q < kNodeStride; ++q) {
        const double t = block_sum<kBlock>(acc[q], lds);
        if (threadIdx.x == 0) part[kNodeStride * blockIdx.x + q] = t;
    }
}

// pass 2 per block: sum (z - m)^2 and 2|z - m| u; m read from device
__global__ __launch_bounds__(kBlock) void k_metrics_centred(int64_t n, const double* __restrict__ z, double c,
                                                            const double* __restrict__ out, double* part) {
    __shared__ double lds[kWavesPerBlock];
    const double m = out[kOutMean];
    int64_t base = static_cast<int64_t>(blockIdx.x) * kNodeTile + threadIdx.x;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < kNodeItems; ++k) {
        int64_t i = base + static_cast<int64_t>(k) * kBlock;
        if (i < n) {
            const double d = z[i] - m;
            a += d * d;
            b += 2.0 * fabs(d) * (z[i] + c);
        }
    }
    a = block_sum<kBlock>(a, lds);
    b = block_sum<kBlock>(b, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// edges: each lane accumulates its own arcs over a light tile or one chunk of
// a heavy row; fixed-order block sums of a d^2, a 2|d|(u_i + u_j), a (u_i + u_j)^2
// upper (undirected graphs): only the arcs (i, j) with j > i, so each edge
// once; the pattern and weights are symmetric (validated at create), so this
// is the same sum as half of the one over all stored arcs, with half the
// gathers.
__global__ __launch_bounds__(kBlock) void k_metrics_edges(TileView tv, const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, const float* __restrict__ w,
                                                          const double* __restrict__ z, double c, int upper,
                                                          double* part) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_z[kWavesPerBlock][64];
    __shared__ double lds[kWavesPerBlock];
    const int wid = wave_id(), lane = lane_id();
    const int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    double acc = 0.0, acc1 = 0.0, acc2 = 0.0;
    auto arc = [&](double zi, int64_t i, int k) {
        const int j = col[k];
        if (upper && j < i) return;
        const double zj = z[j];
        const double d = zi - zj, us = (zi + c) + (zj + c);
        const double a = w ? static_cast<double>(w[k]) : 1.0;
        acc += a * d * d;
        acc1 += a * 2.0 * fabs(d) * us;
        acc2 += a * us * us;
    };
    if (wv < tv.nchunks) {
        const int64_t cc = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[cc]];
        const double zi = z[row];
        const int beg = tv.chunk_beg[cc];
        const int end = min(beg + kArcBudget, row_ptr[row + 1]);
        for (int k = beg + lane; k < end; k += 64) arc(zi, row, k);
    } else if (wv - tv.nchunks < tv.ntiles) {
        const int64_t tix = tv.t0 + (wv - tv.nchunks);
        if (tv.tile_heavy[tix] < 0) {
            const int32_t r0 = tv.tile_start[tix];
            const int nrows = tv.tile_start[tix + 1] - r0;
            if (lane < nrows) s_z[wid][lane] = z[r0 + lane];
            tile_for_each_arc(row_ptr, r0, nrows, s_pre[wid],
                              [&](int k, int slot) { arc(s_z[wid][slot], r0 + slot, k); });
        }
    }
    acc = block_sum<kBlock>(acc, lds);
    acc1 = block_sum<kBlock>(acc1, lds);
    acc2 = block_sum<kBlock>(acc2, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = acc;
        part[3 * blockIdx.x + 1] = acc1;
        part[3 * blockIdx.x + 2] = acc2;
    }
}

// single block: fixed-order sum of `cnt` partials with stride `stride` starting at `off`
__device__ double reduce_parts(const double* part, int64_t cnt, int stride, int off, double* lds) {
    // eight independent sums per thread so that eight loads are in flight,
    // then added in a fixed order
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = threadIdx.x;
    for (; i + 7 * 1024 < cnt; i += 8 * 1024) {
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] += part[(i + u * 1024) * stride + off];
    }
    for (int u = 0; i < cnt; i += 1024, ++u) q[u] += part[i * stride + off];
    double a = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    a = wave_sum(a);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = a;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < 16; ++k) t += lds[k];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(1024) void k_metrics_mean(const double* part, int64_t nb, int64_t n, double* out) {
    __shared__ double lds[16];
    double t[kNodeStride];
    for (int q = 0; q < kNodeStride; ++q) t[q] = reduce_parts(part, nb, kNodeStride, q, lds);
    if (threadIdx.x == 0) {
        const double inv = n ? 1.0 / static_cast<double>(n) : 0.0;
        out[kOutMean] = n ? t[0] / static_cast<double>(n) : 0.0;
        out[kOutC] = t[1];
        out[kOutI] = t[2];
        out[kOutUbar] = t[3] * inv;
        out[kOutC1] = t[4];
        out[kOutI1] = t[5];
        out[kOutQ] = t[6];
    }
}

__global__ __launch_bounds__(1024) void k_metrics_final(const double* part_p, int64_t nbp, const double* part_d,
                                                        int64_t nbd, double* out) {
    __shared__ double lds[16];
    const double p = reduce_parts(part_p, nbp, 2, 0, lds);
    const double p1 = reduce_parts(part_p, nbp, 2, 1, lds);
    const double d = reduce_parts(part_d, nbd, 3, 0, lds);
    const double d1 = reduce_parts(part_d, nbd, 3, 1, lds);
    const double d2 = reduce_parts(part_d, nbd, 3, 2, lds);
    if (threadIdx.x == 0) {
        out[kOutP] = p;
        out[kOutP1] = p1;
        out[kOutD] = d;
        out[kOutD1] = d1;
        out[kOutD2] = d2;
    }
}

// D from per-block sums formed elsewhere (the certificate's gather pass, over
// every stored arc: dscale 0.5 on an undirected graph, where each edge is
// stored twice), P from the centred pass
__global__ __launch_bounds__(1024) void k_measures_final(const double* part_p, int64_t nbp, const double* part_d,
                                                         int64_t nbd, double dscale, double* out) {
    __shared__ double lds[16];
    const double p = reduce_parts(part_p, nbp, 2, 0, lds);
    const double d = reduce_parts(part_d, nbd, 1, 0, lds);
    if (threadIdx.x == 0) {
        out[kOutP] = p;
        out[kOutD] = dscale * d;
    }
}

// ------------------------------------------------------------------ stress
// Per-node stress of Sec. 3.4: (z_i - s_i)^2 + sum_j a_ij (z_i - z_j)^2 over
// row i of A.  Light tiles finish their rows; each heavy-row chunk writes its
// partial sum, and k_stress_heavy adds them in chunk order.
__global__ __launch_bounds__(kBlock) void k_stress_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, const float* __restrict__ w,
                                                         const double* __restrict__ s, const double* __restrict__ z,
                                                         double* stress, double* partial) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    __shared__ double s_z[kWavesPerBlock][64];
    const int wid = wave_id(), lane = lane_id();
    const int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (wv < tv.nchunks) {
        const int64_t c = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[c]];
        const double zi = z[row];
        const int beg = tv.chunk_beg[c];
        const int end = min(beg + kArcBudget, row_ptr[row + 1]);
        const double part = chunk_sum(beg, end, [&](int k) {
            const double d = zi - z[col[k]];
            return (w ? static_cast<double>(w[k]) : 1.0) * d * d;
        });
        if (lane == 0) partial[c] = part;
        return;
    }
    if (wv - tv.nchunks >= tv.ntiles) return;
    const int64_t tix = tv.t0 + (wv - tv.nchunks);
    if (tv.tile_heavy[tix] >= 0) return;  // finished by k_stress_heavy
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    if (lane < nrows) s_z[wid][lane] = z[r0 + lane];
    wave_sync_lds();
    const double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], [&](int k, int slot) {
        const double d = s_z[wid][slot] - z[col[k]];
        return (w ? static_cast<double>(w[k]) : 1.0) * d * d;
    });
    if (lane < nrows) {
        const double d = s_z[wid][lane] - s[r0 + lane];
        stress[r0 + lane] = d * d + sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_stress_heavy(TileView tv, const double* __restrict__ s,
                                                         const double* __restrict__ z,
                                                         const double* __restrict__ partial, double* stress) {
    const int lane = lane_id();
    const int64_t h = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (h >= tv.h1) return;
    double sum = 0.0;
    for (int32_t c = tv.heavy_chunk0[h] + lane; c < tv.heavy_chunk0[h + 1]; c += 64) sum += partial[c];
    sum = wave_sum(sum);
    if (lane == 0) {
        const int32_t row = tv.heavy_row[h];
        const double d = z[row] - s[row];
        stress[row] = d * d + sum;
    }
}

// fixed-order block sums of a node vector
__global__ __launch_bounds__(kBlock) void k_node_sum(int64_t n, const double* __restrict__ x, double* part) {
    __shared__ double lds[kWavesPerBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kNodeTile + threadIdx.x;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < kNodeItems; ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * kBlock;
        if (i < n) a += x[i];
    }
    a = block_sum<kBlock>(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(1024) void k_sum_parts(const double* part, int64_t nb, double* out) {
    __shared__ double lds[16];
    const double t = reduce_parts(part, nb, 1, 0, lds);
    if (threadIdx.x == 0) *out = t;
}

struct StressLayout {
    double* stress; double* partial; double* part; double* out;
};

StressLayout carve_stress(Carver& cv, const fj_graph* g) {
    StressLayout L{};
    L.stress = cv.take<double>(g->n + 1);
    L.partial = cv.take<double>(g->tiles_a.nchunks + 1);
    L.part = cv.take<double>(nblocks_nodes(g->n) + 1);
    L.out = cv.take<double>(1);
    return L;
}

struct MetricsLayout {
    double* part1; double* part2; double* part_d; double* out;
};

MetricsLayout carve_metrics(Carver& cv, const fj_graph* g) {
    const int64_t n = g->n;
    MetricsLayout L{};
    L.part1 = cv.take<double>(kNodeStride * (nblocks_nodes(n) + 1));
    L.part2 = cv.take<double>(2 * (nblocks_nodes(n) + 1));
    L.part_d = cv.take<double>(3 * (nblocks_edges(g) + 1));
    L.out = cv.take<double>(kOutSlots);
    return L;
}

// The measures and the bound sums, into h[kOutSlots] on the host.
fj_status metrics_passes(const fj_graph* g, const double* s, const double* z, double c, const MetricsLayout& L,
                         hipStream_t st, double* h) {
    for (int q = 0; q < kOutSlots; ++q) h[q] = 0.0;
    const int64_t n = g->n;
    if (n == 0) return FJ_OK;
    const unsigned nbn = nblocks_nodes(n), nbt = nblocks_edges(g);
    hipLaunchKernelGGL(k_metrics_nodes, dim3(nbn), dim3(kBlock), 0, st, n, s, z, c, L.part1);
    hipLaunchKernelGGL(k_metrics_edges, dim3(nbt), dim3(kBlock), 0, st, tile_view_all(g->tiles_a), g->row_ptr,
                       g->col, g->w, z, c, g->directed ? 0 : 1, L.part_d);
    hipLaunchKernelGGL(k_metrics_mean, dim3(1), dim3(1024), 0, st, L.part1, static_cast<int64_t>(nbn), n, L.out);
    hipLaunchKernelGGL(k_metrics_centred, dim3(nbn), dim3(kBlock), 0, st, n, z, c, L.out, L.part2);
    hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(1024), 0, st, L.part2, static_cast<int64_t>(nbn), L.part_d,
                       static_cast<int64_t>(nbt), L.out);
    FJ_HIP(hipMemcpyAsync(h, L.out, sizeof(double) * kOutSlots, hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    return FJ_OK;
}

// ------------------------------------------------- allocation-free measures
// For callers that cannot allocate (code under graph capture, serving loops):
// the partial sums of the measures live in this file-scope device array, one
// copy per GPU, instead of a caller workspace.  Host code must never pass the
// array's name to a kernel or copy: it is a host-side stand-in, not a device
// address.  The device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex scratch_mu;
void* scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the current device, looked up once.
fj_status current_scratch(int dev, void** out) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        FJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("fj_metrics_noalloc: hipGetSymbolAddress returned a null address");
            return FJ_ERR_HIP;
        }
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return FJ_OK;
}

size_t metrics_scratch_bytes(const fj_graph* g) {
    Carver cv(nullptr);
    carve_metrics(cv, g);
    return cv.bytes();
}

}  // namespace
}  // namespace fj

using namespace fj;

extern "C" size_t fj_metrics_workspace_bytes(const fj_graph* g) {
    if (!g) return 0;
    Carver cv(nullptr);
    carve_metrics(cv, g);
    size_t cert = certify_ws_bytes(g);  // fj_certify shares this workspace
    return cv.bytes() > cert ? cv.bytes() : cert;
}

namespace fj {

size_t measures_ws_bytes(const fj_graph* g) { return fj_metrics_workspace_bytes(g); }

// fj_metrics without the argument checks, for fj_solve_opts.measures
fj_status measures_full(const fj_graph* g, const double* s, const double* z, void* ws, hipStream_t st,
                        fj_metrics_out* out) {
    Carver cv(ws);
    const MetricsLayout L = carve_metrics(cv, g);
    double h[kOutSlots];
    const fj_status rc = metrics_passes(g, s, z, 0.0, L, st, h);
    if (rc != FJ_OK) return rc;
    *out = fj_metrics_out{h[kOutP], h[kOutD], h[kOutI], h[kOutC], h[kOutMean]};
    return FJ_OK;
}

// The measures with D's per-block sums already formed over every stored arc
// (nbd of them in part_d); the node passes run here.
fj_status measures_with_d(const fj_graph* g, const double* s, const double* z, const double* part_d, int64_t nbd,
                          void* ws, hipStream_t st, fj_metrics_out* out) {
    const int64_t n = g->n;
    if (n == 0) {
        *out = fj_metrics_out{0.0, 0.0, 0.0, 0.0, 0.0};
        return FJ_OK;
    }
    Carver cv(ws);
    const MetricsLayout L = carve_metrics(cv, g);
    const unsigned nbn = nblocks_nodes(n);
    hipLaunchKernelGGL(k_metrics_nodes, dim3(nbn), dim3(kBlock), 0, st, n, s, z, 0.0, L.part1);
    hipLaunchKernelGGL(k_metrics_mean, dim3(1), dim3(1024), 0, st, L.part1, static_cast<int64_t>(nbn), n, L.out);
    hipLaunchKernelGGL(k_metrics_centred, dim3(nbn), dim3(kBlock), 0, st, n, z, 0.0, L.out, L.part2);
    hipLaunchKernelGGL(k_measures_final, dim3(1), dim3(1024), 0, st, L.part2, static_cast<int64_t>(nbn), part_d, nbd,
                       g->directed ? 1.0 : 0.5, L.out);
    double h[kOutSlots];
    FJ_HIP(hipMemcpyAsync(h, L.out, sizeof(double) * kOutSlots, hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    *out = fj_metrics_out{h[kOutP], h[kOutD], h[kOutI], h[kOutC], h[kOutMean]};
    return FJ_OK;
}

}  // namespace fj

extern "C" fj_status fj_metrics(const fj_graph* g, const double* s, const double* z, fj_metrics_out* out, void* ws,
                                size_t ws_bytes, void* stream) {
    if (!g || !out || !ws || ((!s || !z) && g->n > 0)) {
        set_error("fj_metrics: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_metrics_workspace_bytes(g)) {
        set_error("fj_metrics: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    Carver cv(ws);
    const MetricsLayout L = carve_metrics(cv, g);
    double h[kOutSlots];
    const fj_status rc = metrics_passes(g, s, z, 0.0, L, static_cast<hipStream_t>(stream), h);
    if (rc != FJ_OK) return rc;
    out->P = h[kOutP];
    out->D = h[kOutD];
    out->I = h[kOutI];
    out->C = h[kOutC];
    out->mean = h[kOutMean];
    return FJ_OK;
}

extern "C" fj_status fj_metrics_bounds(const fj_graph* g, const double* s, const double* z, double c,
                                       fj_metrics_out* out, fj_metrics_out* bound, double* tau, void* ws,
                                       size_t ws_bytes, void* stream) {
    if (!g || !out || !bound || !ws || ((!s || !z) && g->n > 0)) {
        set_error("fj_metrics_bounds: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!(c >= 0.0) || !std::isfinite(c)) {
        set_error("fj_metrics_bounds: need finite c >= 0");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_metrics_workspace_bytes(g)) {
        set_error("fj_metrics_bounds: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // residual level first (its workspace is reused by the passes after it)
    double t = 0.0;
    if (g->n > 0) {
        const fj_status rc = residual_level(g, s, z, c, ws, ws_bytes, st, &t);
        if (rc != FJ_OK) return rc;
    }
    Carver cv(ws);
    const MetricsLayout L = carve_metrics(cv, g);
    double h[kOutSlots];
    const fj_status rc = metrics_passes(g, s, z, c, L, st, h);
    if (rc != FJ_OK) return rc;
    out->P = h[kOutP];
    out->D = h[kOutD];
    out->I = h[kOutI];
    out->C = h[kOutC];
    out->mean = h[kOutMean];
    if (tau) *tau = t;
    if (!(t < 1.0)) {  // no bound (also for a non-finite level)
        bound->P = bound->D = bound->I = bound->C = bound->mean = INFINITY;
        return FJ_OK;
    }
    const double k = t / (1.0 - t), k2 = k * k;
    bound->C = k * h[kOutC1] + k2 * h[kOutQ];
    bound->I = k * h[kOutI1] + k2 * h[kOutQ];
    bound->P = k * h[kOutP1] + k2 * h[kOutQ];
    bound->D = k * h[kOutD1] + k2 * h[kOutD2];
    bound->mean = k * h[kOutUbar];
    return FJ_OK;
}

extern "C" size_t fj_stress_workspace_bytes(const fj_graph* g) {
    if (!g) return 0;
    Carver cv(nullptr);
    carve_stress(cv, g);
    return cv.bytes();
}

extern "C" fj_status fj_stress(const fj_graph* g, const double* s, const double* z, double* stress, double* total,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!g || !total || !ws || ((!s || !z) && g->n > 0)) {
        set_error("fj_stress: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_stress_workspace_bytes(g)) {
        set_error("fj_stress: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    Carver cv(ws);
    StressLayout L = carve_stress(cv, g);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = g->n;
    double h = 0.0;
    if (n > 0) {
        double* out = stress ? stress : L.stress;
        const TileView tv = tile_view_all(g->tiles_a);
        hipLaunchKernelGGL(k_stress_tiles, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0, st, tv,
                           g->row_ptr, g->col, g->w, s, z, out, L.partial);
        if (tv.h1 > tv.h0)
            hipLaunchKernelGGL(k_stress_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0, st, tv, s, z,
                               L.partial, out);
        const unsigned nbn = nblocks_nodes(n);
        hipLaunchKernelGGL(k_node_sum, dim3(nbn), dim3(kBlock), 0, st, n, out, L.part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, L.part, static_cast<int64_t>(nbn), L.out);
        FJ_HIP(hipMemcpyAsync(&h, L.out, sizeof(double), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
    }
    *total = h;
    return FJ_OK;
}

extern "C" size_t fj_metrics_noalloc_max_bytes(void) { return kStaticScratchBytes; }

extern "C" size_t fj_metrics_noalloc_bytes(const fj_graph* g) { return g ? metrics_scratch_bytes(g) : 0; }

extern "C" fj_status fj_metrics_noalloc(const fj_graph* g, const double* s, const double* z, fj_metrics_out* out,
                                        void* stream) {
    if (!g || !out || ((!s || !z) && g->n > 0)) {
        set_error("fj_metrics_noalloc: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const size_t need = metrics_scratch_bytes(g);
    if (need > kStaticScratchBytes) {
        set_error("fj_metrics_noalloc: the graph's partial sums need " + std::to_string(need) +
                  " bytes, more than the " + std::to_string(kStaticScratchBytes) +
                  "-byte static scratch; use fj_metrics with a workspace");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = -1;
    FJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error("fj_metrics_noalloc: device ordinal out of range");
        return FJ_ERR_UNSUPPORTED;
    }
    if (st) {
        int sdev = -1;
        FJ_HIP(hipStreamGetDevice(st, &sdev));
        if (sdev != dev) {
            set_error("fj_metrics_noalloc: the stream belongs to another device than the current one");
            return FJ_ERR_INVALID_ARGUMENT;
        }
    }
    void* base = nullptr;
    {
        const fj_status rc = current_scratch(dev, &base);
        if (rc != FJ_OK) return rc;
    }
    Carver cv(base);
    const MetricsLayout L = carve_metrics(cv, g);
    double h[kOutSlots];
    const fj_status rc = metrics_passes(g, s, z, 0.0, L, st, h);
    if (rc != FJ_OK) return rc;
    out->P = h[kOutP];
    out->D = h[kOutD];
    out->I = h[kOutI];
    out->C = h[kOutC];
    out->mean = h[kOutMean];
    return FJ_OK;
}
