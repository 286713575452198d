// Relaxation factor from the spectral radius mu = rho((I+D)^{-1} A), by
// Eq. (optimal-omega): omega = 1 + (mu / (1 + sqrt(1 - mu^2)))^2, and the
// paper's own heuristic (Sec. 5.2): try omega from just below 2 downwards in
// fixed steps and keep the one with the fewest updates.
//
// mu by power iteration.  Undirected graphs iterate on the symmetric
// B = (I+D)^{-1/2} A (I+D)^{-1/2}, similar to (I+D)^{-1} A; directed graphs on
// M = (I+D)^{-1} A itself.  Both are nonnegative, so from the positive start
// x0 = 1/sqrt(n) the norms ||B x_k|| (with ||x_k|| = 1) tend to the Perron root.
#include <cmath>
#include <vector>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_tile.h"

namespace fj {
namespace {

constexpr int kNodeItems = 8;
constexpr int kNodeTile = kBlock * kNodeItems;
inline unsigned nblocks_nodes(int64_t n) { return static_cast<unsigned>((n + kNodeTile - 1) / kNodeTile); }
inline unsigned grid1(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// rowscale, colscale from 1 + d; v = colscale / sqrt(n)
__global__ void k_pow_init(int64_t n, int directed, const double* __restrict__ opd, double* rowscale,
                           double* colscale, double* v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double o = opd[i];
    const double r = directed ? 1.0 / o : 1.0 / sqrt(o);
    const double c = directed ? 1.0 : 1.0 / sqrt(o);
    rowscale[i] = r;
    colscale[i] = c;
    v[i] = c / sqrt(static_cast<double>(n));
}

// y_i = rowscale_i * sum_j a_ij v_j over light tiles; heavy-row chunks write partials
__global__ __launch_bounds__(kBlock) void k_pow_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const float* __restrict__ w,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ rowscale, double* y,
                                                      double* partial) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    const int wid = wave_id(), lane = lane_id();
    const int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    auto arc = [&](int k) { return (w ? static_cast<double>(w[k]) : 1.0) * v[col[k]]; };
    if (wv < tv.nchunks) {
        const int64_t c = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[c]];
        const int beg = tv.chunk_beg[c];
        const int end = min(beg + kArcBudget, row_ptr[row + 1]);
        const double part = chunk_sum(beg, end, arc);
        if (lane == 0) partial[c] = part;
        return;
    }
    if (wv - tv.nchunks >= tv.ntiles) return;
    const int64_t tix = tv.t0 + (wv - tv.nchunks);
    if (tv.tile_heavy[tix] >= 0) return;  // finished by k_pow_heavy
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    const double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], arc);
    if (lane < nrows) y[r0 + lane] = rowscale[r0 + lane] * sum;
}

__global__ __launch_bounds__(kBlock) void k_pow_heavy(TileView tv, const double* __restrict__ partial,
                                                      const double* __restrict__ rowscale, double* y) {
    const int lane = lane_id();
    const int64_t h = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (h >= tv.h1) return;
    double sum = 0.0;
    for (int32_t c = tv.heavy_chunk0[h] + lane; c < tv.heavy_chunk0[h + 1]; c += 64) sum += partial[c];
    sum = wave_sum(sum);
    if (lane == 0) {
        const int32_t row = tv.heavy_row[h];
        y[row] = rowscale[row] * sum;
    }
}

// fixed-order block sums of y^2
__global__ __launch_bounds__(kBlock) void k_pow_sq(int64_t n, const double* __restrict__ y, double* part) {
    __shared__ double lds[kWavesPerBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kNodeTile + threadIdx.x;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < kNodeItems; ++k) {
        const int64_t i = base + static_cast<int64_t>(k) * kBlock;
        if (i < n) a += y[i] * y[i];
    }
    a = block_sum<kBlock>(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(1024) void k_pow_norm(const double* __restrict__ part, int64_t nb, double* norm_out) {
    __shared__ double lds[16];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += 1024) a += part[i];
    a = wave_sum(a);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += lds[k];
        *norm_out = sqrt(t);
    }
}

// v = colscale * y / ||y||  (a zero vector stays zero)
__global__ void k_pow_scale(int64_t n, const double* __restrict__ y, const double* __restrict__ colscale,
                            const double* __restrict__ norm, double* v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nv = *norm;
    v[i] = nv > 0.0 ? colscale[i] * y[i] / nv : 0.0;
}

struct OmegaLayout {
    double* rowscale; double* colscale; double* v; double* y; double* partial; double* part; double* norms;
};

constexpr int kMaxPowIters = 100000;

OmegaLayout carve_omega(Carver& cv, const fj_graph* g) {
    OmegaLayout L{};
    const int64_t n = g->n;
    L.rowscale = cv.take<double>(n + 1);
    L.colscale = cv.take<double>(n + 1);
    L.v = cv.take<double>(n + 1);
    L.y = cv.take<double>(n + 1);
    L.partial = cv.take<double>(g->tiles_a.nchunks + 1);
    L.part = cv.take<double>(nblocks_nodes(n) + 1);
    L.norms = cv.take<double>(kMaxPowIters);
    return L;
}

}  // namespace
}  // namespace fj

using namespace fj;

extern "C" double fj_optimal_omega(double mu) {
    if (!(mu >= 0.0)) return 1.0;
    if (mu >= 1.0) return 2.0;
    const double q = mu / (1.0 + std::sqrt(1.0 - mu * mu));
    return 1.0 + q * q;
}

extern "C" size_t fj_omega_workspace_bytes(const fj_graph* g) {
    if (!g) return 0;
    Carver cv(nullptr);
    carve_omega(cv, g);
    return cv.bytes();
}

extern "C" fj_status fj_estimate_omega(const fj_graph* g, int32_t max_iters, double tol, double* mu, double* omega,
                                       int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
    if (!g || !mu || !omega || !ws || max_iters < 1 || max_iters > kMaxPowIters || !(tol >= 0.0)) {
        set_error("fj_estimate_omega: bad argument (max_iters must be in [1, 100000], tol >= 0)");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_omega_workspace_bytes(g)) {
        set_error("fj_estimate_omega: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = g->n;
    if (n == 0 || g->nnz == 0) {  // (I+D)^{-1} A = 0
        *mu = 0.0;
        *omega = 1.0;
        if (iters) *iters = 0;
        return FJ_OK;
    }
    Carver cv(ws);
    OmegaLayout L = carve_omega(cv, g);
    const int bs = 256;
    const TileView tv = tile_view_all(g->tiles_a);
    const unsigned nbn = nblocks_nodes(n);
    hipLaunchKernelGGL(k_pow_init, dim3(grid1(n, bs)), dim3(bs), 0, st, n, g->directed, g->opd, L.rowscale,
                       L.colscale, L.v);
    const int check = 10;
    std::vector<double> h(check);
    int it = 0;
    double est = 0.0;
    while (it < max_iters) {
        const int todo = std::min(check, max_iters - it);
        for (int b = 0; b < todo; ++b) {
            hipLaunchKernelGGL(k_pow_tiles, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0, st, tv,
                               g->row_ptr, g->col, g->w, L.v, L.rowscale, L.y, L.partial);
            if (tv.h1 > tv.h0)
                hipLaunchKernelGGL(k_pow_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0, st, tv,
                                   L.partial, L.rowscale, L.y);
            hipLaunchKernelGGL(k_pow_sq, dim3(nbn), dim3(kBlock), 0, st, n, L.y, L.part);
            hipLaunchKernelGGL(k_pow_norm, dim3(1), dim3(1024), 0, st, L.part, static_cast<int64_t>(nbn),
                               L.norms + it + b);
            hipLaunchKernelGGL(k_pow_scale, dim3(grid1(n, bs)), dim3(bs), 0, st, n, L.y, L.colscale,
                               L.norms + it + b, L.v);
        }
        FJ_HIP(hipMemcpyAsync(h.data(), L.norms + it, sizeof(double) * todo, hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
        const double prev = est;
        est = h[todo - 1];
        it += todo;
        if (!std::isfinite(est)) {
            set_error("fj_estimate_omega: non-finite power iterate");
            return FJ_ERR_NOT_CONVERGED;
        }
        if (it > check && std::fabs(est - prev) <= tol * est) break;
    }
    *mu = est;
    *omega = fj_optimal_omega(est);
    if (iters) *iters = it;
    return FJ_OK;
}
