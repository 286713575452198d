// Learned warm start: a two-layer message-passing network that proposes a
// starting estimate z0 for the push.  Not part of the paper's method: by
// Lemma 4 any start is valid (r = s - (I+L) z0) and by Lemma 7 the residual
// certificate decides the result, so the network only changes how long the
// sweeps run.  fj_jacobi_steps implements the FJ update of Eq. (1) itself and
// serves as the untrained control.
//
// Network (hidden width 64, BF16 storage, FP32 accumulation on MFMA):
//   X0 = [s, nbr(s), log1p d, log1p din, 1/(1+d), mean s, 1, 0]
//   H1 = relu([X0 | nbr(X0)] W1 + b1),  H2 = relu([H1 | nbr(H1)] W2 + b2)
//   z0 = min s + (max s - min s) sigmoid(H2 u + c0)
// with nbr(x)_v = sum_j a_vj x_j / d_v.  Parameters are one flat FP32 vector:
// W1 (16x64), b1 (64), W2 (128x64), b2 (64), u (64), c0 (1).
#include <cmath>
#include <cstring>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_tile.h"

namespace fj {
namespace {

constexpr int kF = 8;     // input features
constexpr int kH = 64;    // hidden width
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 9280, kOffU = 9344, kOffC0 = 9408;
constexpr int kNParams = 9409;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

inline unsigned g1d(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// -------------------------------------------------------------- scalars
// [0] sum s, [1] min s, [2] max s over n, per block then one block
__global__ __launch_bounds__(256) void k_s_stats(int64_t n, const double* __restrict__ s, double* part) {
    __shared__ double a[4], b[4], c[4];
    double sm = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256) {
        double v = s[i];
        sm += v; mn = fmin(mn, v); mx = fmax(mx, v);
    }
    sm = wave_sum(sm);
    for (int o = 32; o > 0; o >>= 1) { mn = fmin(mn, __shfl_xor(mn, o, 64)); mx = fmax(mx, __shfl_xor(mx, o, 64)); }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) { a[w] = sm; b[w] = mn; c[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0, m1 = INFINITY, m2 = -INFINITY;
        for (int k = 0; k < 4; ++k) { t += a[k]; m1 = fmin(m1, b[k]); m2 = fmax(m2, c[k]); }
        part[3 * blockIdx.x + 0] = t; part[3 * blockIdx.x + 1] = m1; part[3 * blockIdx.x + 2] = m2;
    }
}
__global__ void k_s_stats_final(int nb, int64_t n, const double* __restrict__ part, double* out) {
    if (threadIdx.x != 0) return;
    double t = 0, m1 = INFINITY, m2 = -INFINITY;
    for (int k = 0; k < nb; ++k) { t += part[3 * k]; m1 = fmin(m1, part[3 * k + 1]); m2 = fmax(m2, part[3 * k + 2]); }
    out[0] = n ? t / static_cast<double>(n) : 0.0;  // mean
    out[1] = m1;
    out[2] = m2;
}

// ----------------------------------------------------------- row sums
// out[i] = sum over CSR row i of f(k); light tiles here, heavy rows by chunk
// partials + k_rowsum_heavy (fixed order).
template <int MODE>  // 0: sum a_ij s_j (CSR(A)); 1: sum of weights (in-degree over CSR(A^T))
__global__ __launch_bounds__(kBlock) void k_rowsum_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, const float* __restrict__ w,
                                                         const double* __restrict__ x, double* partial, double* out) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    auto f = [&](int k) {
        double a = w ? static_cast<double>(w[k]) : 1.0;
        if constexpr (MODE == 0) return a * x[col[k]];
        return a;
    };
    if (wv < tv.nchunks) {
        const int64_t c = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[c]];
        const int beg = tv.chunk_beg[c];
        double sum = chunk_sum(beg, min(beg + kArcBudget, row_ptr[row + 1]), f);
        if (lane == 0) partial[c] = sum;
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], f);
    if (lane < nrows) out[r0 + lane] = sum;
}

__global__ __launch_bounds__(kBlock) void k_rowsum_heavy(TileView tv, const double* __restrict__ partial, double* out) {
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (hh >= tv.h1) return;
    double sum = 0.0;
    for (int32_t q = tv.heavy_chunk0[hh] + lane; q < tv.heavy_chunk0[hh + 1]; q += 64) sum += partial[q];
    sum = wave_sum(sum);
    if (lane == 0) out[tv.heavy_row[hh]] = sum;
}

// --------------------------------------------------------------- features
__global__ void k_features(int64_t n, const double* __restrict__ s, const double* __restrict__ ws_sum,
                           const double* __restrict__ opd, const double* __restrict__ din,
                           const double* __restrict__ stats, uint16_t* X0) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = opd[i] - 1.0;
    const double nb = d > 0.0 ? ws_sum[i] / d : 0.0;
    float f[kF] = {static_cast<float>(s[i]), static_cast<float>(nb), static_cast<float>(log1p(d)),
                   static_cast<float>(log1p(din[i])), static_cast<float>(1.0 / (1.0 + d)),
                   static_cast<float>(stats[0]), 1.0f, 0.0f};
    for (int q = 0; q < kF; ++q) X0[i * kF + q] = f2bf(f[q]);
}

__global__ void k_inv_deg(int64_t n, const double* __restrict__ opd, float* invd) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = opd[i] - 1.0;
    invd[i] = d > 0.0 ? static_cast<float>(1.0 / d) : 0.0f;
}

// ------------------------------------------------------------ aggregation
// M_v = sum_j a_vj X_j / d_v over CSR(A) rows, X bf16 [n][D] -> M bf16 [n][D].
// Every lane loads 16 bytes (8 features) of a gathered row, so one arc takes
// D/8 lanes.  Rows longer than kArcBudget are done by k_agg_heavy (one
// 1024-thread block per row); the light kernels skip them.
struct Acc8 {
    float v[8];
};
__device__ __forceinline__ void acc8_add(Acc8& acc, float a, uint4 x) {
    const uint32_t q[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc.v[2 * t] += a * bf2f(static_cast<uint16_t>(q[t] & 0xffffu));
        acc.v[2 * t + 1] += a * bf2f(static_cast<uint16_t>(q[t] >> 16));
    }
}
__device__ __forceinline__ uint4 acc8_pack(const Acc8& acc, float sc) {
    uint32_t q[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        q[t] = static_cast<uint32_t>(f2bf(acc.v[2 * t] * sc)) | (static_cast<uint32_t>(f2bf(acc.v[2 * t + 1] * sc)) << 16);
    return uint4{q[0], q[1], q[2], q[3]};
}

// lanes of one wave in groups of D/8; group g takes arcs b + start + g, + stride, ...
template <int D>
__device__ __forceinline__ void agg_accum(int b, int e, int lane, const int32_t* __restrict__ col,
                                          const float* __restrict__ w, const uint16_t* __restrict__ X, int start,
                                          int stride, Acc8& acc) {
    constexpr int L = D / 8;  // lanes per arc
    const int sub = lane / L, part = lane % L;
    for (int k = b + start + sub; k < e; k += stride) {
        const int j = col[k];
        const float a = w ? w[k] : 1.0f;
        acc8_add(acc, a, reinterpret_cast<const uint4*>(X + static_cast<int64_t>(j) * D)[part]);
    }
}

// fold the 64 / (D/8) arc groups of a wave, fixed order; lanes < D/8 hold the row
template <int D>
__device__ __forceinline__ void agg_fold(Acc8& acc) {
#pragma unroll
    for (int o = D / 8; o < 64; o <<= 1)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc.v[q] += __shfl_xor(acc.v[q], o, 64);
}

// D = 8: eight lanes per row (16 bytes per arc, lane p of a row takes its
// arcs p, p + 8, ...), eight consecutive rows per wave, grid-stride over the
// groups of eight rows.  The eight partial sums of a row are folded in a
// fixed order.
__global__ __launch_bounds__(kBlock) void k_agg_rows8(int64_t n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, const float* __restrict__ w,
                                                     const float* __restrict__ invd, const uint16_t* __restrict__ X,
                                                     uint16_t* M) {
    const int lane = lane_id(), p = lane & 7;
    const int64_t groups = (n + 7) / 8;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    for (int64_t gi = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6); gi < groups;
         gi += stride) {
        const int64_t i = gi * 8 + (lane >> 3);
        int b = 0, e = 0;
        if (i < n) {
            b = row_ptr[i];
            e = row_ptr[i + 1];
            if (e - b > kArcBudget) e = b;  // heavy: k_agg_heavy
        }
        Acc8 acc{};
        for (int k = b + p; k < e; k += 8) {
            const int j = col[k];
            const float a = w ? w[k] : 1.0f;
            acc8_add(acc, a, reinterpret_cast<const uint4*>(X)[j]);
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc.v[q] += __shfl_xor(acc.v[q], o, 64);
        if (p == 0 && i < n && row_ptr[i + 1] - row_ptr[i] <= kArcBudget)
            reinterpret_cast<uint4*>(M)[i] = acc8_pack(acc, invd[i]);
    }
}

// D = 64: a wave per row, 8 lanes per arc (one 128-byte line), 8 arcs per step;
// grid-stride over rows.
__global__ __launch_bounds__(kBlock) void k_agg_rows64(int64_t n, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const float* __restrict__ w,
                                                      const float* __restrict__ invd, const uint16_t* __restrict__ X,
                                                      uint16_t* M) {
    const int lane = lane_id();
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6); i < n; i += stride) {
        const int b = row_ptr[i], e = row_ptr[i + 1];
        if (e - b > kArcBudget) continue;  // uniform across the wave
        Acc8 acc{};
        agg_accum<kH>(b, e, lane, col, w, X, 0, 8, acc);
        agg_fold<kH>(acc);
        if (lane < 8) reinterpret_cast<uint4*>(M + i * kH)[lane] = acc8_pack(acc, invd[i]);
    }
}

template <int D>
__global__ __launch_bounds__(1024) void k_agg_heavy(TileView tv, const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, const float* __restrict__ w,
                                                    const float* __restrict__ invd, const uint16_t* __restrict__ X,
                                                    uint16_t* M) {
    constexpr int L = D / 8, G = 64 / L;  // lanes per arc, arcs per wave step
    __shared__ Acc8 part[16][L];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int32_t i = tv.heavy_row[tv.h0 + blockIdx.x];
    const int b = row_ptr[i], e = row_ptr[i + 1];
    Acc8 acc{};
    agg_accum<D>(b, e, lane, col, w, X, wid * G, 16 * G, acc);
    agg_fold<D>(acc);
    if (lane < L) part[wid][lane] = acc;
    __syncthreads();
    if (wid == 0 && lane < L) {
        Acc8 t{};
        for (int v = 0; v < 16; ++v)
#pragma unroll
            for (int q = 0; q < 8; ++q) t.v[q] += part[v][lane].v[q];
        reinterpret_cast<uint4*>(M + static_cast<int64_t>(i) * D)[lane] = acc8_pack(t, invd[i]);
    }
}

// grid for the grid-stride kernels: enough waves to fill every CU, no more
// than the work needs
inline unsigned stride_blocks(int64_t waves, int per_cu = 16) {
    const int64_t cap = 256 * static_cast<int64_t>(per_cu);  // blocks of 4 waves per CU
    const int64_t need = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min(need, cap)));
}

// Backward of the aggregation: out_j = sum over u with a_uj > 0 of
// (a_uj / d_u) G_u, i.e. a gather over row j of CSR(A^T).  G is the right half
// (columns 64..127) of dA2 (FP32, row stride 128).  Fused with the rest of
// layer 1's backward: dY1_j = (dA2_j[0:64] + out_j) * [H1_j > 0].
__global__ __launch_bounds__(kBlock) void k_aggT_light(int64_t n, const int32_t* __restrict__ t_row_ptr,
                                                       const int32_t* __restrict__ t_col, const float* __restrict__ t_w,
                                                       const float* __restrict__ invd, const float* __restrict__ dA2,
                                                       const uint16_t* __restrict__ H1, float* dY1) {
    const int lane = lane_id();
    const int64_t j = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) >> 6;
    if (j >= n) return;
    const int b = t_row_ptr[j], e = t_row_ptr[j + 1];
    if (e - b > kArcBudget) return;
    float acc = 0.f;
    for (int k = b; k < e; ++k) {
        const int u = t_col[k];
        const float a = (t_w ? t_w[k] : 1.0f) * invd[u];
        acc += a * dA2[static_cast<int64_t>(u) * 128 + 64 + lane];
    }
    const float g = dA2[j * 128 + lane] + acc;
    dY1[j * kH + lane] = bf2f(H1[j * kH + lane]) > 0.f ? g : 0.f;
}

__global__ __launch_bounds__(1024) void k_aggT_heavy(TileView tv, const int32_t* __restrict__ t_row_ptr,
                                                     const int32_t* __restrict__ t_col, const float* __restrict__ t_w,
                                                     const float* __restrict__ invd, const float* __restrict__ dA2,
                                                     const uint16_t* __restrict__ H1, float* dY1) {
    __shared__ float sacc[16][64];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int32_t j = tv.heavy_row[tv.h0 + blockIdx.x];
    const int b = t_row_ptr[j], e = t_row_ptr[j + 1];
    float acc = 0.f;
    for (int k = b + wid; k < e; k += 16) {
        const int u = t_col[k];
        const float a = (t_w ? t_w[k] : 1.0f) * invd[u];
        acc += a * dA2[static_cast<int64_t>(u) * 128 + 64 + lane];
    }
    sacc[wid][lane] = acc;
    __syncthreads();
    if (wid == 0) {
        float t = 0.f;
        for (int v = 0; v < 16; ++v) t += sacc[v][lane];
        const float g = dA2[static_cast<int64_t>(j) * 128 + lane] + t;
        dY1[static_cast<int64_t>(j) * kH + lane] = bf2f(H1[static_cast<int64_t>(j) * kH + lane]) > 0.f ? g : 0.f;
    }
}

// ------------------------------------------------------------------ GEMM
// Y[16 rows x N] per wave on v_mfma_f32_16x16x16_bf16: A = [A_left | A_right]
// (bf16, widths KL and KR, row-major), W (bf16) read from LDS as Wt[j][k].
// Lane l supplies A[row l%16][k 4(l/16)..+3] and Wt[col l%16][k 4(l/16)..+3];
// it receives D[rows 4(l/16)+q][col l%16].
// MODE 0: H = relu(Y + b) stored bf16 [n][N]
// MODE 1: H2 = relu(Y + b) stored bf16; o = H2 u + c0; z0 = lo + (hi-lo) sigmoid(o)
// MODE 2: as 1 without storing H2 (inference)
// MODE 3: Y stored FP32 [n][N] (backward: dA = dY W^T; W given as [N][K])
template <int KL, int KR, int N, int MODE>
__global__ __launch_bounds__(kBlock) void k_gemm(int64_t n, const uint16_t* __restrict__ Al,
                                                 const uint16_t* __restrict__ Ar, const uint16_t* __restrict__ W,
                                                 const float* __restrict__ bias, const float* __restrict__ u,
                                                 const float* __restrict__ c0, const double* __restrict__ stats,
                                                 uint16_t* Hout, float* Yout, float* o_out, double* z0) {
    constexpr int K = KL + KR;
    static_assert(K % 16 == 0 && N % 16 == 0 && KL % 4 == 0, "tile shapes");
    __shared__ uint16_t Wt[N][K + 4];
    for (int idx = threadIdx.x; idx < N * K; idx += kBlock) {  // coalesced reads of W
        if constexpr (MODE == 3) Wt[idx / K][idx % K] = W[idx];
        else Wt[idx % N][idx / N] = W[idx];
    }
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int li = lane & 15, lk = (lane >> 4) * 4;
    // grid-stride over 16-row tiles, so every block loads W once
    const int64_t tile_stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock * 16;
    for (int64_t row0 = (static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid) * 16; row0 < n;
         row0 += tile_stride) {
        const int64_t ar = min(row0 + li, n - 1);
        f32x4 acc[N / 16];
#pragma unroll
        for (int t = 0; t < N / 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) {
            const int k = ks * 16 + lk;
            bf16x4 a;
            if (k < KL) a = *reinterpret_cast<const bf16x4*>(Al + ar * KL + k);
            else a = *reinterpret_cast<const bf16x4*>(Ar + ar * KR + (k - KL));
#pragma unroll
            for (int t = 0; t < N / 16; ++t) {
                const bf16x4 bv = *reinterpret_cast<const bf16x4*>(&Wt[t * 16 + li][k]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[t], 0, 0, 0);
            }
        }
        if constexpr (MODE == 3) {
#pragma unroll
            for (int t = 0; t < N / 16; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t r = row0 + lk + q;
                    if (r < n) Yout[r * N + t * 16 + li] = acc[t][q];
                }
            continue;
        }
        float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < N / 16; ++t) {
            const int j = t * 16 + li;
            const float bj = bias[j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = row0 + lk + q;
                const float h = fmaxf(acc[t][q] + bj, 0.f);
                const uint16_t hb = f2bf(h);
                if constexpr (MODE == 0 || MODE == 1)
                    if (r < n) Hout[r * N + j] = hb;
                if constexpr (MODE == 1 || MODE == 2) p[q] += bf2f(hb) * u[j];
            }
        }
        if constexpr (MODE == 1 || MODE == 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) p[q] += __shfl_xor(p[q], o, 64);
            if (li == 0) {
                const double lo = stats[1], hi = stats[2];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t r = row0 + lk + q;
                    if (r < n) {
                        const float o = p[q] + c0[0];
                        if (o_out) o_out[r] = o;
                        const double sg = 1.0 / (1.0 + exp(-static_cast<double>(o)));
                        z0[r] = lo + (hi - lo) * sg;
                    }
                }
            }
        }
    }  // row tiles
}

// -------------------------------------------------- readout backward + loss
// do = (2/n)(z0 - z*) (hi-lo) sg(1-sg);  dY2 = do u * [H2 > 0] (FP32 and bf16);
// per-block partial of sum (z0 - z*)^2.
__global__ __launch_bounds__(kBlock) void k_readout_bwd(int64_t n, const double* __restrict__ z0,
                                                        const double* __restrict__ zt, const float* __restrict__ o,
                                                        const double* __restrict__ stats, const float* __restrict__ u,
                                                        const uint16_t* __restrict__ H2, float* dout, float* dY2,
                                                        uint16_t* dY2b, double* loss_part) {
    __shared__ double lds[kWavesPerBlock];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;  // a wave per row
    double l2 = 0.0;
    if (r < n) {
        const double diff = z0[r] - zt[r];
        const double sg = 1.0 / (1.0 + exp(-static_cast<double>(o[r])));
        const float dor = static_cast<float>(2.0 * diff / static_cast<double>(n) * (stats[2] - stats[1]) * sg * (1.0 - sg));
        if (lane == 0) { dout[r] = dor; l2 = diff * diff; }
        const float g = bf2f(H2[r * kH + lane]) > 0.f ? dor * u[lane] : 0.f;
        dY2[r * kH + lane] = g;
        dY2b[r * kH + lane] = f2bf(g);
    }
    l2 = block_sum<kBlock>(l2, lds);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = l2;
}

// ---------------------------------------------------- A^T B reductions
// out[k][j] = sum_rows A'[row][k] B[row][j] with A' = [A_left | A_right | 1]
// (bf16 inputs; the trailing ones column yields the bias gradient), B FP32
// [n][N].  Blocks own row ranges; each thread owns fixed (k, j) outputs; the
// per-block partials are summed in block order by k_atb_final.
constexpr int kAtbRows = 64;
constexpr int kAtbBlocks = 256;

template <int KL, int KR, int N>
__global__ __launch_bounds__(256) void k_atb(int64_t n, const uint16_t* __restrict__ Al,
                                             const uint16_t* __restrict__ Ar, const float* __restrict__ B, float* part) {
    constexpr int K1 = KL + KR + 1;
    constexpr int OUT = K1 * N;
    constexpr int PER = (OUT + 255) / 256;
    __shared__ float sa[kAtbRows][K1];
    __shared__ float sb[kAtbRows][N];
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.f;
    const int64_t per_block = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r_begin = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t r_end = min(n, r_begin + per_block);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kAtbRows) {
        const int rows = static_cast<int>(min<int64_t>(kAtbRows, r_end - r0));
        for (int idx = threadIdx.x; idx < kAtbRows * K1; idx += 256) {
            const int rr = idx / K1, k = idx % K1;
            float v = 0.f;
            if (rr < rows) {
                const int64_t r = r0 + rr;
                if (k < KL) v = bf2f(Al[r * KL + k]);
                else if (k < KL + KR) v = bf2f(Ar[r * KR + (k - KL)]);
                else v = 1.0f;
            }
            sa[rr][k] = v;
        }
        for (int idx = threadIdx.x; idx < kAtbRows * N; idx += 256) {
            const int rr = idx / N, j = idx % N;
            sb[rr][j] = rr < rows ? B[(r0 + rr) * N + j] : 0.f;
        }
        __syncthreads();
        for (int rr = 0; rr < rows; ++rr) {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int o = threadIdx.x + q * 256;
                if (o < OUT) acc[q] += sa[rr][o / N] * sb[rr][o % N];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int o = threadIdx.x + q * 256;
        if (o < OUT) part[static_cast<int64_t>(blockIdx.x) * OUT + o] = acc[q];
    }
}

__global__ void k_atb_final(int nb, int out_count, const float* __restrict__ part, float* grad) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= out_count) return;
    float t = 0.f;
    for (int b = 0; b < nb; ++b) t += part[static_cast<int64_t>(b) * out_count + o];
    grad[o] = t;
}

__global__ void k_loss_final(int nb, int64_t n, const double* __restrict__ part, float* loss) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[b];
    *loss = static_cast<float>(t / static_cast<double>(n));
}

// ------------------------------------------------------- weights and Adam
__global__ void k_weights_bf16(const float* __restrict__ p, uint16_t* w1, uint16_t* w2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 16 * kH) w1[i] = f2bf(p[kOffW1 + i]);
    if (i < 128 * kH) w2[i] = f2bf(p[kOffW2 + i]);
}

__global__ void k_adam(int count, float* p, const float* __restrict__ g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------- FJ iteration
// Eq. (1): z_i <- (s_i + sum_j a_ij z_j) / (1 + sum_j a_ij), synchronously.
__global__ __launch_bounds__(kBlock) void k_fj_step_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, const float* __restrict__ w,
                                                          const double* __restrict__ s, const double* __restrict__ zin,
                                                          const double* __restrict__ opd, double* partial, double* zout) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    const int wid = threadIdx.x >> 6, lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    auto f = [&](int k) { return (w ? static_cast<double>(w[k]) : 1.0) * zin[col[k]]; };
    if (wv < tv.nchunks) {
        const int64_t c = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[c]];
        const int beg = tv.chunk_beg[c];
        double sum = chunk_sum(beg, min(beg + kArcBudget, row_ptr[row + 1]), f);
        if (lane == 0) partial[c] = sum;
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], f);
    if (lane < nrows) zout[r0 + lane] = (s[r0 + lane] + sum) / opd[r0 + lane];
}

__global__ __launch_bounds__(kBlock) void k_fj_step_heavy(TileView tv, const double* __restrict__ s,
                                                          const double* __restrict__ opd,
                                                          const double* __restrict__ partial, double* zout) {
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (hh >= tv.h1) return;
    double sum = 0.0;
    for (int32_t q = tv.heavy_chunk0[hh] + lane; q < tv.heavy_chunk0[hh + 1]; q += 64) sum += partial[q];
    sum = wave_sum(sum);
    if (lane == 0) {
        const int32_t i = tv.heavy_row[hh];
        zout[i] = (s[i] + sum) / opd[i];
    }
}

// ---------------------------------------------------------------- layout
struct NetLayout {
    double* stats_part; double* stats; double* rs; double* din; double* partial; float* invd;
    uint16_t* X0; uint16_t* M0; uint16_t* H1; uint16_t* M1; uint16_t* H2;
    float* o; double* z0; float* dout; float* dY2; uint16_t* dY2b; float* dA2; float* dY1;
    float* atb_part; double* loss_part; float* grad; uint16_t* w1b; uint16_t* w2b;
};

constexpr int kStatBlocks = 256;

NetLayout carve_net(Carver& cv, const fj_graph* g, bool training) {
    NetLayout L{};
    const int64_t n = g->n;
    L.stats_part = cv.take<double>(3 * kStatBlocks);
    L.stats = cv.take<double>(4);
    L.rs = cv.take<double>(n);
    L.din = cv.take<double>(n);
    L.partial = cv.take<double>(std::max(g->tiles_a.nchunks, g->tiles_t.nchunks) + 1);
    L.invd = cv.take<float>(n);
    L.X0 = cv.take<uint16_t>(n * kF);
    L.M0 = cv.take<uint16_t>(n * kF);
    L.H1 = cv.take<uint16_t>(n * kH);
    L.M1 = cv.take<uint16_t>(n * kH);
    L.w1b = cv.take<uint16_t>(16 * kH);
    L.w2b = cv.take<uint16_t>(128 * kH);
    L.o = cv.take<float>(n);
    if (training) {
        L.H2 = cv.take<uint16_t>(n * kH);
        L.z0 = cv.take<double>(n);
        L.dout = cv.take<float>(n);
        L.dY2 = cv.take<float>(n * kH);
        L.dY2b = cv.take<uint16_t>(n * kH);
        L.dA2 = cv.take<float>(n * 128);
        L.dY1 = cv.take<float>(n * kH);
        L.atb_part = cv.take<float>(static_cast<int64_t>(kAtbBlocks) * 129 * kH);
        L.loss_part = cv.take<double>(waves_to_blocks(n) + 1);
        L.grad = cv.take<float>(kNParams + 3);
    }
    return L;
}

// forward up to (and including) layer 2; training keeps H2 and o
fj_status net_forward(const fj_graph* g, const double* s, const float* params, double* z0, const NetLayout& L,
                      bool training, hipStream_t st) {
    const int64_t n = g->n;
    const int bs = 256;
    hipLaunchKernelGGL(k_weights_bf16, dim3(g1d(128 * kH, 256)), dim3(256), 0, st, params, L.w1b, L.w2b);
    hipLaunchKernelGGL(k_s_stats, dim3(kStatBlocks), dim3(256), 0, st, n, s, L.stats_part);
    hipLaunchKernelGGL(k_s_stats_final, dim3(1), dim3(64), 0, st, kStatBlocks, n, L.stats_part, L.stats);
    {   // neighbour sum of s over CSR(A)
        TileView tv = tile_view_all(g->tiles_a);
        hipLaunchKernelGGL(k_rowsum_tiles<0>, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0, st, tv,
                           g->row_ptr, g->col, g->w, s, L.partial, L.rs);
        if (tv.h1 > tv.h0)
            hipLaunchKernelGGL(k_rowsum_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0, st, tv,
                               L.partial, L.rs);
    }
    {   // in-degree: row sums of CSR(A^T)
        TileView tv = tile_view_all(g->tiles_t);
        hipLaunchKernelGGL(k_rowsum_tiles<1>, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0, st, tv,
                           g->t_row_ptr, g->t_col, g->t_w, static_cast<const double*>(nullptr), L.partial, L.din);
        if (tv.h1 > tv.h0)
            hipLaunchKernelGGL(k_rowsum_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0, st, tv,
                               L.partial, L.din);
    }
    hipLaunchKernelGGL(k_inv_deg, dim3(g1d(n, bs)), dim3(bs), 0, st, n, g->opd, L.invd);
    hipLaunchKernelGGL(k_features, dim3(g1d(n, bs)), dim3(bs), 0, st, n, s, L.rs, g->opd, L.din, L.stats, L.X0);
    const TileView ta = tile_view_all(g->tiles_a);
    hipLaunchKernelGGL(k_agg_rows8, dim3(stride_blocks(g1d(n, 8))), dim3(kBlock), 0, st, n, g->row_ptr, g->col,
                       g->w, L.invd, L.X0, L.M0);
    if (ta.h1 > ta.h0)
        hipLaunchKernelGGL(k_agg_heavy<kF>, dim3(ta.h1 - ta.h0), dim3(1024), 0, st, ta, g->row_ptr, g->col, g->w,
                           L.invd, L.X0, L.M0);
    const unsigned nb_gemm = stride_blocks(g1d(n, 16), 8);
    hipLaunchKernelGGL((k_gemm<kF, kF, kH, 0>), dim3(nb_gemm), dim3(kBlock), 0, st, n, L.X0, L.M0, L.w1b,
                       params + kOffB1, params + kOffU, params + kOffC0, L.stats, L.H1, static_cast<float*>(nullptr),
                       static_cast<float*>(nullptr), static_cast<double*>(nullptr));
    hipLaunchKernelGGL(k_agg_rows64, dim3(stride_blocks(n)), dim3(kBlock), 0, st, n, g->row_ptr, g->col, g->w,
                       L.invd, L.H1, L.M1);
    if (ta.h1 > ta.h0)
        hipLaunchKernelGGL(k_agg_heavy<kH>, dim3(ta.h1 - ta.h0), dim3(1024), 0, st, ta, g->row_ptr, g->col, g->w,
                           L.invd, L.H1, L.M1);
    if (training)
        hipLaunchKernelGGL((k_gemm<kH, kH, kH, 1>), dim3(nb_gemm), dim3(kBlock), 0, st, n, L.H1, L.M1, L.w2b,
                           params + kOffB2, params + kOffU, params + kOffC0, L.stats, L.H2,
                           static_cast<float*>(nullptr), L.o, z0);
    else
        hipLaunchKernelGGL((k_gemm<kH, kH, kH, 2>), dim3(nb_gemm), dim3(kBlock), 0, st, n, L.H1, L.M1, L.w2b,
                           params + kOffB2, params + kOffU, params + kOffC0, L.stats,
                           static_cast<uint16_t*>(nullptr), static_cast<float*>(nullptr), L.o, z0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "warm-start forward");
    return FJ_OK;
}

fj_status net_grad(const fj_graph* g, const double* s, const double* zt, const float* params, const NetLayout& L,
                   float* grad, float* loss, hipStream_t st) {
    const int64_t n = g->n;
    fj_status rc = net_forward(g, s, params, L.z0, L, true, st);
    if (rc) return rc;
    const unsigned nbw = waves_to_blocks(n);
    hipLaunchKernelGGL(k_readout_bwd, dim3(nbw), dim3(kBlock), 0, st, n, L.z0, zt, L.o, L.stats, params + kOffU,
                       L.H2, L.dout, L.dY2, L.dY2b, L.loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, static_cast<int>(nbw), n, L.loss_part, loss);
    // du, dc0 = [H2 | 1]^T do
    hipLaunchKernelGGL((k_atb<kH, 0, 1>), dim3(kAtbBlocks), dim3(256), 0, st, n, L.H2,
                       static_cast<const uint16_t*>(nullptr), L.dout, L.atb_part);
    hipLaunchKernelGGL(k_atb_final, dim3(1), dim3(128), 0, st, kAtbBlocks, kH + 1, L.atb_part, grad + kOffU);
    // dW2, db2 = [H1 | M1 | 1]^T dY2
    hipLaunchKernelGGL((k_atb<kH, kH, kH>), dim3(kAtbBlocks), dim3(256), 0, st, n, L.H1, L.M1, L.dY2, L.atb_part);
    hipLaunchKernelGGL(k_atb_final, dim3(g1d(129 * kH, 256)), dim3(256), 0, st, kAtbBlocks, 129 * kH, L.atb_part,
                       grad + kOffW2);
    // dA2 = dY2 W2^T (MFMA; W2 read as [N=128][K=64])
    const unsigned nb_gemm = stride_blocks(g1d(n, 16), 8);
    hipLaunchKernelGGL((k_gemm<kH, 0, 128, 3>), dim3(nb_gemm), dim3(kBlock), 0, st, n, L.dY2b,
                       static_cast<const uint16_t*>(nullptr), L.w2b, static_cast<const float*>(nullptr),
                       static_cast<const float*>(nullptr), static_cast<const float*>(nullptr),
                       static_cast<const double*>(nullptr), static_cast<uint16_t*>(nullptr), L.dA2,
                       static_cast<float*>(nullptr), static_cast<double*>(nullptr));
    // dY1 = (dA2[:, :64] + nbr^T(dA2[:, 64:])) * [H1 > 0]
    hipLaunchKernelGGL(k_aggT_light, dim3(g1d(n * 64, kBlock)), dim3(kBlock), 0, st, n, g->t_row_ptr, g->t_col,
                       g->t_w, L.invd, L.dA2, L.H1, L.dY1);
    const TileView tt = tile_view_all(g->tiles_t);
    if (tt.h1 > tt.h0)
        hipLaunchKernelGGL(k_aggT_heavy, dim3(tt.h1 - tt.h0), dim3(1024), 0, st, tt, g->t_row_ptr, g->t_col, g->t_w,
                           L.invd, L.dA2, L.H1, L.dY1);
    // dW1, db1 = [X0 | M0 | 1]^T dY1
    hipLaunchKernelGGL((k_atb<kF, kF, kH>), dim3(kAtbBlocks), dim3(256), 0, st, n, L.X0, L.M0, L.dY1, L.atb_part);
    hipLaunchKernelGGL(k_atb_final, dim3(g1d(17 * kH, 256)), dim3(256), 0, st, kAtbBlocks, 17 * kH, L.atb_part,
                       grad + kOffW1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "warm-start backward");
    return FJ_OK;
}

}  // namespace
}  // namespace fj

using namespace fj;

extern "C" int32_t fj_wsnet_param_count(void) { return kNParams; }

extern "C" size_t fj_wsnet_workspace_bytes(const fj_graph* g, int32_t training) {
    if (!g) return 0;
    Carver cv(nullptr);
    carve_net(cv, g, training != 0);
    return cv.bytes();
}

static fj_status net_args_ok(const fj_graph* g, const void* a, const void* b, void* ws, size_t ws_bytes, bool training) {
    if (!g || !a || !b || !ws || g->n <= 0) {
        set_error("warm-start network: null argument or empty graph");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_wsnet_workspace_bytes(g, training ? 1 : 0)) {
        set_error("warm-start network: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    return FJ_OK;
}

extern "C" fj_status fj_wsnet_forward(const fj_graph* g, const double* s, const float* params, double* z0, void* ws,
                                      size_t ws_bytes, void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, false);
    if (rc) return rc;
    if (!z0) {
        set_error("fj_wsnet_forward: z0 is NULL");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    NetLayout L = carve_net(cv, g, false);
    return net_forward(g, s, params, z0, L, false, static_cast<hipStream_t>(stream));
}

extern "C" fj_status fj_wsnet_grad(const fj_graph* g, const double* s, const double* z_target, const float* params,
                                   float* grad, float* loss, void* ws, size_t ws_bytes, void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, true);
    if (rc) return rc;
    if (!z_target || !grad || !loss) {
        set_error("fj_wsnet_grad: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    NetLayout L = carve_net(cv, g, true);
    return net_grad(g, s, z_target, params, L, grad, loss, static_cast<hipStream_t>(stream));
}

extern "C" fj_status fj_wsnet_train_step(const fj_graph* g, const double* s, const double* z_target, float* params,
                                         float* adam_m, float* adam_v, int32_t step, float lr, float* loss, void* ws,
                                         size_t ws_bytes, void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, true);
    if (rc) return rc;
    if (!z_target || !adam_m || !adam_v || !loss || step < 1 || !(lr > 0.f)) {
        set_error("fj_wsnet_train_step: bad argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    NetLayout L = carve_net(cv, g, true);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = net_grad(g, s, z_target, params, L, L.grad, loss, st);
    if (rc) return rc;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, static_cast<float>(step)), c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam, dim3(g1d(kNParams, 256)), dim3(256), 0, st, kNParams, params, L.grad, adam_m, adam_v,
                       lr, b1, b2, 1e-8f, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "adam");
    return FJ_OK;
}

extern "C" size_t fj_jacobi_workspace_bytes(const fj_graph* g) {
    if (!g) return 0;
    Carver cv(nullptr);
    cv.take<double>(g->n);
    cv.take<double>(g->tiles_a.nchunks + 1);
    return cv.bytes();
}

extern "C" fj_status fj_jacobi_steps(const fj_graph* g, const double* s, double* z, int32_t steps, void* ws,
                                     size_t ws_bytes, void* stream) {
    if (!g || !s || !z || steps < 0 || !ws || ws_bytes < fj_jacobi_workspace_bytes(g)) {
        set_error("fj_jacobi_steps: bad argument or workspace too small");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g->n == 0 || steps == 0) return FJ_OK;
    Carver cv(ws);
    double* tmp = cv.take<double>(g->n);
    double* partial = cv.take<double>(g->tiles_a.nchunks + 1);
    const TileView tv = tile_view_all(g->tiles_a);
    double* src = z;
    double* dst = tmp;
    for (int it = 0; it < steps; ++it) {
        hipLaunchKernelGGL(k_fj_step_tiles, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0, st, tv,
                           g->row_ptr, g->col, g->w, s, src, g->opd, partial, dst);
        if (tv.h1 > tv.h0)
            hipLaunchKernelGGL(k_fj_step_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0, st, tv, s,
                               g->opd, partial, dst);
        std::swap(src, dst);
    }
    if (src != z) FJ_HIP(hipMemcpyAsync(z, src, sizeof(double) * g->n, hipMemcpyDeviceToDevice, st));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "jacobi");
    return FJ_OK;
}
