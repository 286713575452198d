// Learned warm start: a two-layer message-passing network that proposes a
// starting estimate z0 for the push.  Not part of the paper's method: by
// Lemma 4 any start is valid (r = s - (I+L) z0) and by Lemma 7 the residual
// certificate decides the result, so the network only changes how long the
// sweeps run.  fj_jacobi_steps implements the FJ update of Eq. (1) itself and
// serves as the untrained control.
//
// Network (hidden width 64, BF16 operands on MFMA, FP32 accumulation):
//   ns = nbr(s),  z1 = (s + d ns) / (1 + d)      (one step of Eq. (1) from s)
//   X0 = [s, ns, z1, log1p d, 1/(1+d), mean s, 1, 0]
//   H1 = relu(X0 W1 + b1)                        layer 1 (its message: s)
//   P  = H1 Wp,  M = nbr(P)                      layer 2's 16-wide message
//   H2 = relu([H1 | M] W2 + b2)                  layer 2
//   z0 = min s + (max s - min s) sigmoid(H2 u + c0)
// with nbr(x)_v = sum_j a_vj x_j / d_v.  Parameters are one flat FP32 vector:
// W1 (8x64), b1 (64), Wp (64x16), W2 (80x64), b2 (64), u (64), c0 (1).
//
// Every dense product runs on v_mfma_f32_16x16x16_bf16 over 16-row tiles, one
// tile per wave step: the per-node layers (X0 -> H1 -> P and [H1|M] -> H2 ->
// z0) and, in training, the weight gradients (X0^T dY1, H1^T dP, [H1|M]^T dY2)
// and the products with transposed weights.  The gathers are the only
// passes over the arcs: the neighbour sum of s, the 16-wide message over
// CSR(A) forward and its transpose over CSR(A^T) backward.  The network never
// stores H1, H2 or dY2: each tile kernel recomputes layer 1 from X0.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_tile.h"

namespace fj {
namespace {

constexpr int kF = 8;     // input features
constexpr int kH = 64;    // hidden width
constexpr int kMsg = 16;  // width of layer 2's message
constexpr int kK2 = kH + kMsg;  // inputs of layer 2
constexpr int kOffW1 = 0, kOffB1 = 512, kOffWp = 576, kOffW2 = 1600, kOffB2 = 6720, kOffU = 6784, kOffC0 = 6848;
constexpr int kNParams = 6849;
static_assert(kOffB1 == kF * kH && kOffWp == kOffB1 + kH && kOffW2 == kOffWp + kH * kMsg &&
                  kOffB2 == kOffW2 + kK2 * kH && kOffU == kOffB2 + kH && kOffC0 == kOffU + kH && kNParams == kOffC0 + 1,
              "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even (gfx950 converts in hardware: v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

inline unsigned g1d(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 v;
    v[0] = static_cast<short>(f2bf(a));
    v[1] = static_cast<short>(f2bf(b));
    v[2] = static_cast<short>(f2bf(c));
    v[3] = static_cast<short>(f2bf(d));
    return v;
}
__device__ __forceinline__ bf16x4 lds4(const uint16_t* p) {  // 8-byte aligned LDS read
    return *reinterpret_cast<const bf16x4*>(p);
}
constexpr f32x4 kZero4 = {0.f, 0.f, 0.f, 0.f};



// ------------------------------------------------------------ aggregation
// BF16 rows of 8 features, accumulated in FP32: 16 bytes per lane and arc.
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

// grid for the grid-stride kernels: enough waves to fill every CU, no more
// than the work needs
inline unsigned stride_blocks(int64_t waves, int per_cu = 16) {
    const int64_t cap = 256 * static_cast<int64_t>(per_cu);  // blocks of 4 waves per CU
    const int64_t need = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min(need, cap)));
}


// ------------------------------------------------- per-call node passes
// One pass over the nodes: per-block sum, min and max of s, the FP32 copy of
// s the neighbour sums gather, and 1/d (0 where d = 0) for the means.
__global__ __launch_bounds__(256) void k_s_prep(int64_t n, const double* __restrict__ s,
                                                const double* __restrict__ opd, double* part, float* s32,
                                                float* invd) {
    __shared__ double a[4], b[4], c[4];
    double sm = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const double v = s[i], d = opd[i] - 1.0;
        sm += v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
        s32[i] = static_cast<float>(v);
        invd[i] = d > 0.0 ? static_cast<float>(1.0 / d) : 0.0f;
    }
    sm = wave_sum(sm);
    for (int o = 32; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    const int w = wave_id();
    if (lane_id() == 0) { a[w] = sm; b[w] = mn; c[w] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0, m1 = INFINITY, m2 = -INFINITY;
        for (int k = 0; k < 4; ++k) { t += a[k]; m1 = fmin(m1, b[k]); m2 = fmax(m2, c[k]); }
        part[3 * blockIdx.x + 0] = t; part[3 * blockIdx.x + 1] = m1; part[3 * blockIdx.x + 2] = m2;
    }
}
// mean, min, max from the block partials: one wave, fixed order
__global__ void k_s_final(int nb, int64_t n, const double* __restrict__ part, double* out) {
    const int lane = lane_id();
    double t = 0, m1 = INFINITY, m2 = -INFINITY;
    for (int k = lane; k < nb; k += 64) {
        t += part[3 * k];
        m1 = fmin(m1, part[3 * k + 1]);
        m2 = fmax(m2, part[3 * k + 2]);
    }
    t = wave_sum(t);
    for (int o = 32; o > 0; o >>= 1) {
        m1 = fmin(m1, __shfl_xor(m1, o, 64));
        m2 = fmax(m2, __shfl_xor(m2, o, 64));
    }
    if (lane == 0) {
        out[0] = n ? t / static_cast<double>(n) : 0.0;
        out[1] = m1;
        out[2] = m2;
    }
}

// rs_i = sum_j a_ij s_j over CSR(A) from the FP32 copy of s, by the
// merge-path tiles of CSR(A): a wave takes a tile of up to 64 light rows and
// streams its arcs in order, four 64-arc chunks in flight, the per-row sums by
// a fixed-order segmented scan (FP64, rounded to FP32 once); heavy tiles are
// left to k_nbr_chunks
__global__ __launch_bounds__(kBlock) void k_nbr_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, const float* __restrict__ w,
                                                     const float* __restrict__ s32, float* rs) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    const int wid = wave_id(), lane = lane_id();
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (t >= tv.ntiles) return;
    const int64_t tix = tv.t0 + t;
    if (tv.tile_heavy[tix] >= 0) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    const double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], [&](int k) {
        const double a = w ? static_cast<double>(w[k]) : 1.0;
        return a * static_cast<double>(s32[col[k]]);
    });
    if (lane < nrows) rs[r0 + lane] = static_cast<float>(sum);
}
// Heavy rows of CSR(A) (more than kArcBudget arcs) in 256-arc chunks, a wave
// per chunk: partial sums per chunk, then k_nbr_combine adds a row's chunks in
// chunk order
__global__ __launch_bounds__(kBlock) void k_nbr_chunks(TileView tv, const int32_t* __restrict__ col,
                                                      const float* __restrict__ w, const float* __restrict__ s32,
                                                      float* partial) {
    const int lane = lane_id();
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (c >= tv.nchunks) return;
    const int64_t cidx = tv.c0 + c;
    const int beg = tv.chunk_beg[cidx], end = tv.chunk_end[cidx];
    float acc = 0.f;
    for (int k = beg + lane; k < end; k += 64) acc += (w ? w[k] : 1.0f) * s32[col[k]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) partial[cidx] = acc;
}
__global__ __launch_bounds__(kBlock) void k_nbr_combine(TileView tv, const float* __restrict__ partial, float* rs) {
    const int lane = lane_id();
    const int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (hh >= tv.h1) return;
    float t = 0.f;
    for (int32_t q = tv.heavy_chunk0[hh] + lane; q < tv.heavy_chunk0[hh + 1]; q += 64) t += partial[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) rs[tv.heavy_row[hh]] = t;
}

// ------------------------------------------------------ message aggregation
// M_v = sum_j a_vj P_j / d_v for the 16-wide BF16 message P over CSR(A): 32
// bytes per arc, two lanes per arc (16 bytes each), eight lanes per row (four
// arcs in flight), eight rows per wave, grid-stride over groups of eight
// rows.  The four arc groups of a row are folded in a fixed order.  Rows
// longer than kArcBudget are left to k_agg16_chunks.
__global__ __launch_bounds__(kBlock) void k_agg_rows16(int64_t n, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const float* __restrict__ w,
                                                      const float* __restrict__ invd, const uint16_t* __restrict__ X,
                                                      uint16_t* M) {
    const int lane = lane_id(), p = lane & 7, sub = p >> 1, half = p & 1;
    const int64_t groups = (n + 7) / 8;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    for (int64_t gi = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id(); gi < groups;
         gi += stride) {
        const int64_t i = gi * 8 + (lane >> 3);
        int b = 0, e = 0;
        if (i < n) {
            b = row_ptr[i];
            e = row_ptr[i + 1];
            if (e - b > kArcBudget) e = b;  // heavy: k_agg16_chunks
        }
        Acc8 acc{};
        // each lane's next column index loads while its current row is gathered
        int k = b + sub;
        int j = k < e ? col[k] : 0;
        float a = k < e ? (w ? w[k] : 1.0f) : 0.0f;
        while (k < e) {
            const uint4 x = reinterpret_cast<const uint4*>(X)[2 * static_cast<int64_t>(j) + half];
            const int kn = k + 4;
            const int jn = kn < e ? col[kn] : 0;
            const float an = kn < e ? (w ? w[kn] : 1.0f) : 0.0f;
            acc8_add(acc, a, x);
            k = kn;
            j = jn;
            a = an;
        }
#pragma unroll
        for (int o = 2; o < 8; o <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc.v[q] += __shfl_xor(acc.v[q], o, 64);
        if (sub == 0 && i < n && row_ptr[i + 1] - row_ptr[i] <= kArcBudget)
            reinterpret_cast<uint4*>(M)[2 * i + half] = acc8_pack(acc, invd[i]);
    }
}

// Heavy rows of the 16-wide aggregation in 256-arc chunks: a wave per chunk
// (two lanes per arc, 32 arcs per step) writes 16 FP32 partial sums; then
// k_agg16_combine adds a row's chunks in chunk order and scales by 1/d.
__global__ __launch_bounds__(kBlock) void k_agg16_chunks(TileView tv, const int32_t* __restrict__ col,
                                                        const float* __restrict__ w, const uint16_t* __restrict__ X,
                                                        float* partial) {
    const int lane = lane_id(), half = lane & 1, sub = lane >> 1;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (c >= tv.nchunks) return;
    const int64_t cidx = tv.c0 + c;
    const int beg = tv.chunk_beg[cidx], end = tv.chunk_end[cidx];
    Acc8 acc{};
    for (int k = beg + sub; k < end; k += 32) {
        const int j = col[k];
        acc8_add(acc, w ? w[k] : 1.0f, reinterpret_cast<const uint4*>(X)[2 * static_cast<int64_t>(j) + half]);
    }
#pragma unroll
    for (int o = 2; o < 64; o <<= 1)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc.v[q] += __shfl_xor(acc.v[q], o, 64);
    if (sub == 0)
#pragma unroll
        for (int q = 0; q < 8; ++q) partial[cidx * kMsg + 8 * half + q] = acc.v[q];
}
__global__ __launch_bounds__(kBlock) void k_agg16_combine(TileView tv, const float* __restrict__ partial,
                                                         const float* __restrict__ invd, uint16_t* M) {
    const int lane = lane_id();
    const int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave_id();
    if (hh >= tv.h1 || lane >= kMsg) return;
    float t = 0.f;
    for (int32_t q = tv.heavy_chunk0[hh]; q < tv.heavy_chunk0[hh + 1]; ++q) t += partial[static_cast<int64_t>(q) * kMsg + lane];
    const int32_t i = tv.heavy_row[hh];
    M[static_cast<int64_t>(i) * kMsg + lane] = f2bf(t * invd[i]);
}

// Backward of the aggregation: dP_j = sum over v with a_vj > 0 of
// (a_vj / d_v) dM_v, a gather over row j of CSR(A^T) of 16-wide FP32 rows.
// Sixteen lanes per row (one feature each), four rows per wave; rows longer
// than kArcBudget are left to k_aggT16_heavy.
__global__ __launch_bounds__(kBlock) void k_aggT16_light(int64_t n, const int32_t* __restrict__ t_row_ptr,
                                                        const int32_t* __restrict__ t_col,
                                                        const float* __restrict__ t_w, const float* __restrict__ invd,
                                                        const float* __restrict__ dM, float* dP) {
    const int lane = lane_id(), f = lane & 15;
    const int64_t j = ((static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) >> 4);
    if (j >= n) return;
    const int b = t_row_ptr[j], e = t_row_ptr[j + 1];
    if (e - b > kArcBudget) return;
    float acc = 0.f;
    for (int k = b; k < e; ++k) {
        const int v = t_col[k];
        acc += (t_w ? t_w[k] : 1.0f) * invd[v] * dM[static_cast<int64_t>(v) * kMsg + f];
    }
    dP[j * kMsg + f] = acc;
}

// one 1024-thread block per heavy row of CSR(A^T): 64 groups of 16 lanes
// stride over its arcs, then the groups are added in a fixed order
__global__ __launch_bounds__(1024) void k_aggT16_heavy(TileView tv, const int32_t* __restrict__ t_row_ptr,
                                                      const int32_t* __restrict__ t_col, const float* __restrict__ t_w,
                                                      const float* __restrict__ invd, const float* __restrict__ dM,
                                                      float* dP) {
    __shared__ float sacc[64][kMsg];
    const int grp = threadIdx.x >> 4, f = threadIdx.x & 15;
    const int32_t j = tv.heavy_row[tv.h0 + blockIdx.x];
    const int b = t_row_ptr[j], e = t_row_ptr[j + 1];
    float acc = 0.f;
    for (int k = b + grp; k < e; k += 64) {
        const int v = t_col[k];
        acc += (t_w ? t_w[k] : 1.0f) * invd[v] * dM[static_cast<int64_t>(v) * kMsg + f];
    }
    sacc[grp][f] = acc;
    __syncthreads();
    if (threadIdx.x < kMsg) {
        float t = 0.f;
        for (int g = 0; g < 64; ++g) t += sacc[g][f];
        dP[static_cast<int64_t>(j) * kMsg + f] = t;
    }
}

// ------------------------------------------------------------ tile kernels
// A wave takes 16 consecutive rows at a time.  v_mfma_f32_16x16x16_bf16:
// lane l (li = l % 16, kq = l / 16) supplies A[row li][k 4kq..4kq+3] and
// B[k 4kq..4kq+3][col li] and receives D[rows 4kq..4kq+3][col li].  D's
// layout is also the A operand of the transposed product (A^T with rows of
// the tile as k), so the weight gradients take layer outputs straight from
// registers.  Weights live in LDS as BF16, transposed where they are B.
constexpr int kW1S = 16 + 4;  // padded row strides (multiples of 4: 8-byte reads)
constexpr int kHS = kH + 4;
constexpr int kW2S = kK2 + 4;
constexpr int kMS = kMsg + 4;

struct NetW {  // forward weights of one block
    uint16_t w1t[kH][kW1S];    // w1t[n][k] = W1[k][n], k < 8 (k 8..15 zero)
    uint16_t wpt[kMsg][kHS];   // wpt[j][m] = Wp[m][j]
    uint16_t w2t[kH][kW2S];    // w2t[n][k] = W2[k][n]
};
struct NetWB {  // extra weights of the backward (row-major)
    uint16_t w2r[kK2][kHS];    // W2[k][n]
    uint16_t wpr[kH][kMS];     // Wp[m][j]
};

__device__ void load_weights(const float* __restrict__ p, NetW& W) {
    for (int i = threadIdx.x; i < kH * 16; i += blockDim.x) {
        const int nn = i / 16, k = i % 16;
        W.w1t[nn][k] = k < kF ? f2bf(p[kOffW1 + k * kH + nn]) : 0;
    }
    for (int i = threadIdx.x; i < kMsg * kH; i += blockDim.x) {
        const int j = i / kH, m = i % kH;
        W.wpt[j][m] = f2bf(p[kOffWp + m * kMsg + j]);
    }
    for (int i = threadIdx.x; i < kH * kK2; i += blockDim.x) {
        const int nn = i / kK2, k = i % kK2;
        W.w2t[nn][k] = f2bf(p[kOffW2 + k * kH + nn]);
    }
}
__device__ void load_weights_bwd(const float* __restrict__ p, NetWB& B) {
    for (int i = threadIdx.x; i < kK2 * kH; i += blockDim.x) B.w2r[i / kH][i % kH] = f2bf(p[kOffW2 + i]);
    for (int i = threadIdx.x; i < kH * kMsg; i += blockDim.x) B.wpr[i / kMsg][i % kMsg] = f2bf(p[kOffWp + i]);
}

struct NetIn {
    int64_t n;
    const double* s;
    const float* rs;      // sum_j a_ij s_j
    const double* opd;    // 1 + d
    const double* stats;  // mean, min, max of s
    const float* p;       // parameters (FP32)
    double rel_floor;     // loss weights 1 / (z + rel_floor)^2 when > 0, else 1
};

// X0 of row r: [s, ns, z1, log1p d, 1/(1+d), mean s, 1, 0], in FP32 (the
// MFMA takes them in BF16)
// a row's inputs to the features: s, 1 + d and the neighbour sum of s
struct RowIn {
    float s, opd, rs;
};
__device__ __forceinline__ RowIn row_in(const NetIn& I, int64_t r) {
    return RowIn{static_cast<float>(I.s[r]), static_cast<float>(I.opd[r]), I.rs[r]};
}
__device__ __forceinline__ void features8_from(const NetIn& I, const RowIn& x, float* f) {
    const float sv = x.s, o = x.opd, d = o - 1.0f, rsv = x.rs;
    const float inv = 1.0f / o;
    f[0] = sv;
    f[1] = d > 0.0f ? rsv / d : 0.0f;
    f[2] = (sv + rsv) * inv;
    f[3] = log1pf(d);
    f[4] = inv;
    f[5] = static_cast<float>(I.stats[0]);
    f[6] = 1.0f;
    f[7] = 0.0f;
}
__device__ __forceinline__ void features8(const NetIn& I, int64_t r, float* f) { features8_from(I, row_in(I, r), f); }

// Layer 1 of the tile at row0: y (D layout) = X0 W1 + b1, h = BF16 relu(y)
// (D layout), and h into the wave's LDS tile Hs[row][unit].
__device__ __forceinline__ void tile_layer1(const NetIn& I, const NetW& W, int64_t row0, int li, int kq, f32x4 y[4],
                                            float h[4][4], uint16_t (*Hs)[kHS]) {
    const int64_t r = min(row0 + li, I.n - 1);
    float f[8];
    features8(I, r, f);
    const bf16x4 a = kq == 0 ? pack4(f[0], f[1], f[2], f[3]) : kq == 1 ? pack4(f[4], f[5], f[6], f[7])
                                                                       : pack4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        y[t] = mfma16(a, lds4(&W.w1t[16 * t + li][4 * kq]), kZero4);
        const float bj = I.p[kOffB1 + 16 * t + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            y[t][q] += bj;
            const uint16_t hb = f2bf(fmaxf(y[t][q], 0.f));
            h[t][q] = bf2f(hb);
            Hs[4 * kq + q][16 * t + li] = hb;
        }
    }
}

// Layer 2 of the tile: y2 (D layout) = [H1 | M] W2 + b2, H1 from Hs
__device__ __forceinline__ void tile_layer2(const NetIn& I, const NetW& W, const uint16_t* __restrict__ M,
                                            int64_t row0, int li, int kq, const uint16_t (*Hs)[kHS], f32x4 y2[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) y2[t] = kZero4;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const bf16x4 a = lds4(&Hs[li][16 * ks + 4 * kq]);
#pragma unroll
        for (int t = 0; t < 4; ++t) y2[t] = mfma16(a, lds4(&W.w2t[16 * t + li][16 * ks + 4 * kq]), y2[t]);
    }
    const int64_t r = min(row0 + li, I.n - 1);
    const bf16x4 am = *reinterpret_cast<const bf16x4*>(M + r * kMsg + 4 * kq);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        y2[t] = mfma16(am, lds4(&W.w2t[16 * t + li][kH + 4 * kq]), y2[t]);
        const float bj = I.p[kOffB2 + 16 * t + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) y2[t][q] += bj;
    }
}

// o for rows 4kq..4kq+3 of the tile (in all 16 lanes of the kq group), from
// H2 = relu(y2) rounded to BF16 (h2, D layout)
__device__ __forceinline__ void tile_readout(const NetIn& I, const f32x4 y2[4], int li, float o[4], float h2[4][4]) {
    float pq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float uj = I.p[kOffU + 16 * t + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            h2[t][q] = bfround(fmaxf(y2[t][q], 0.f));
            pq[q] += h2[t][q] * uj;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) pq[q] += __shfl_xor(pq[q], off, 64);
    const float c0 = I.p[kOffC0];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = pq[q] + c0;
}

// grid-stride tile kernels: at most `cap` blocks, about one resident round
// (k_net_l1: 7 waves per SIMD at its register count, k_net_l2: 3)
inline unsigned fwd_blocks(int64_t n, int64_t cap = 1024) {
    const int64_t tiles = (n + 15) / 16;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(cap, (tiles + kWavesPerBlock - 1) / kWavesPerBlock)));
}
inline unsigned bwd_blocks(int64_t n) {
    const int64_t tiles = (n + 15) / 16;
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(256, (tiles + kWavesPerBlock - 1) / kWavesPerBlock)));
}

// The forward in transposed form: H^T = W^T X^T puts the tile's rows on the
// MFMA's n axis, so lane (li, kq) receives row li's units 16t + 4kq .. +3 --
// exactly the B operand (row li, four consecutive k) of the next product.
// Activations never leave registers.
// Layer 1 of the tile at row0 in this form: h[t][q] = H1[row li][16t + 4kq + q]
// (BF16-rounded); y1 before the relu.
__device__ __forceinline__ void tile_layer1_t(const NetIn& I, const NetW& W, const RowIn& x, int li, int kq,
                                              float y1[4][4], float h[4][4]) {
    float f[8];
    features8_from(I, x, f);
    const bf16x4 b = kq == 0 ? pack4(f[0], f[1], f[2], f[3]) : kq == 1 ? pack4(f[4], f[5], f[6], f[7])
                                                                       : pack4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 y = mfma16(lds4(&W.w1t[16 * t + li][4 * kq]), b, kZero4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            y1[t][q] = y[q] + I.p[kOffB1 + 16 * t + 4 * kq + q];
            h[t][q] = bfround(fmaxf(y1[t][q], 0.f));
        }
    }
}

// P = H1 Wp (BF16 [n][16]); in transposed form lane (li, kq) gets row li's
// message entries 4kq .. 4kq+3 and stores them as one 8-byte word
__global__ __launch_bounds__(kBlock) void k_net_l1(NetIn I, uint16_t* __restrict__ P) {
    __shared__ NetW W;
    load_weights(I.p, W);
    __syncthreads();
    const int wid = wave_id(), lane = lane_id(), li = lane & 15, kq = lane >> 4;
    const int64_t tiles = (I.n + 15) / 16;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    int64_t tt = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    // each tile's row inputs load while the tile before it computes
    RowIn x = tt < tiles ? row_in(I, min(tt * 16 + li, I.n - 1)) : RowIn{0.f, 1.f, 0.f};
    for (; tt < tiles; tt += stride) {
        const int64_t row0 = tt * 16, tn = tt + stride;
        const RowIn xn = tn < tiles ? row_in(I, min(tn * 16 + li, I.n - 1)) : RowIn{0.f, 1.f, 0.f};
        float y1[4][4], h[4][4];
        tile_layer1_t(I, W, x, li, kq, y1, h);
        x = xn;
        f32x4 pt = kZero4;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            pt = mfma16(lds4(&W.wpt[li][16 * ks + 4 * kq]), pack4(h[ks][0], h[ks][1], h[ks][2], h[ks][3]), pt);
        const int64_t r = row0 + li;
        if (r < I.n) *reinterpret_cast<bf16x4*>(P + r * kMsg + 4 * kq) = pack4(pt[0], pt[1], pt[2], pt[3]);
    }
}

// z0 = lo + (hi - lo) sigmoid(o), o = H2 u + c0, H2 = relu([H1 | M] W2 + b2)
__global__ __launch_bounds__(kBlock) void k_net_l2(NetIn I, const uint16_t* __restrict__ M, double* __restrict__ z0) {
    __shared__ NetW W;
    load_weights(I.p, W);
    __syncthreads();
    const int wid = wave_id(), lane = lane_id(), li = lane & 15, kq = lane >> 4;
    const double lo = I.stats[1], hi = I.stats[2];
    const float c0 = I.p[kOffC0];
    const int64_t tiles = (I.n + 15) / 16;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    int64_t tt = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    // each tile's row inputs and message load while the tile before it computes
    auto msg = [&](int64_t t) {
        return *reinterpret_cast<const bf16x4*>(M + min(t * 16 + li, I.n - 1) * kMsg + 4 * kq);
    };
    RowIn x = RowIn{0.f, 1.f, 0.f};
    bf16x4 bm{};
    if (tt < tiles) {
        x = row_in(I, min(tt * 16 + li, I.n - 1));
        bm = msg(tt);
    }
    for (; tt < tiles; tt += stride) {
        const int64_t row0 = tt * 16, tn = tt + stride;
        RowIn xn = RowIn{0.f, 1.f, 0.f};
        bf16x4 bmn{};
        if (tn < tiles) {
            xn = row_in(I, min(tn * 16 + li, I.n - 1));
            bmn = msg(tn);
        }
        float y1[4][4], h[4][4];
        tile_layer1_t(I, W, x, li, kq, y1, h);
        bf16x4 bh[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) bh[ks] = pack4(h[ks][0], h[ks][1], h[ks][2], h[ks][3]);
        float o = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 y2 = kZero4;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) y2 = mfma16(lds4(&W.w2t[16 * t + li][16 * ks + 4 * kq]), bh[ks], y2);
            y2 = mfma16(lds4(&W.w2t[16 * t + li][kH + 4 * kq]), bm, y2);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int unit = 16 * t + 4 * kq + q;
                o += bfround(fmaxf(y2[q] + I.p[kOffB2 + unit], 0.f)) * I.p[kOffU + unit];
            }
        }
        o += __shfl_xor(o, 16, 64);
        o += __shfl_xor(o, 32, 64);
        if (kq == 0 && row0 + li < I.n)
            z0[row0 + li] = lo + (hi - lo) / (1.0 + exp(-static_cast<double>(o + c0)));
        x = xn;
        bm = bmn;
    }
}

// Per-wave partial gradients: [W2 | b2 | u | c0] (5249 floats, the parameter
// layout from W2 on) and [W1 | b1 | Wp] (1600 floats, the layout up to W2).
constexpr int kPart2 = kK2 * kH + kH + kH + 1;
constexpr int kPart1 = kF * kH + kH + kH * kMsg;
static_assert(kPart1 == kOffW2 && kOffW2 + kPart2 == kNParams, "partial layouts");

// The layer-2 part of one tile for the backward: recomputes the forward,
// returns dO (per row 4kq+q, 0 beyond n), dY2 (D layout) and writes dY2 as
// BF16 into Ds[row][unit]; also the squared error of rows in this lane (li 0).
__device__ __forceinline__ void tile_bwd_top(const NetIn& I, const NetW& W, const uint16_t* __restrict__ M,
                                             const double* __restrict__ zt, int64_t row0, int li, int kq,
                                             uint16_t (*Hs)[kHS], uint16_t (*Ds)[kHS], f32x4 y[4], float h[4][4],
                                             float h2[4][4], float dO[4], float dy[4][4], double* sq) {
    f32x4 y2[4];
    float o[4];
    tile_layer1(I, W, row0, li, kq, y, h, Hs);
    wave_sync_lds();
    tile_layer2(I, W, M, row0, li, kq, Hs, y2);
    tile_readout(I, y2, li, o, h2);
    const double lo = I.stats[1], hi = I.stats[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + 4 * kq + q;
        dO[q] = 0.f;
        if (r < I.n) {
            const double sg = 1.0 / (1.0 + exp(-static_cast<double>(o[q])));
            const double diff = lo + (hi - lo) * sg - zt[r];
            const double wv = I.rel_floor > 0.0 ? 1.0 / ((zt[r] + I.rel_floor) * (zt[r] + I.rel_floor)) : 1.0;
            dO[q] = static_cast<float>(2.0 / static_cast<double>(I.n) * wv * diff * (hi - lo) * sg * (1.0 - sg));
            if (li == 0) *sq += wv * diff * diff;
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float uj = I.p[kOffU + 16 * t + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dy[t][q] = y2[t][q] > 0.f ? dO[q] * uj : 0.f;
            Ds[4 * kq + q][16 * t + li] = f2bf(dy[t][q]);
        }
    }
    wave_sync_lds();
}

// Layer 2's gradients ([H1 | M]^T dY2, sums of dY2, H2^T dO, sum dO, the
// loss) and dM = dY2 W2[64:80]^T (FP32 [n][16]).
__global__ __launch_bounds__(kBlock) void k_net_bwd2(NetIn I, const uint16_t* __restrict__ M,
                                                     const double* __restrict__ zt, float* __restrict__ dM,
                                                     float* __restrict__ part, double* __restrict__ loss_part) {
    __shared__ NetW W;
    __shared__ NetWB WB;
    __shared__ uint16_t Hs[kWavesPerBlock][16][kHS];
    __shared__ uint16_t Ds[kWavesPerBlock][16][kHS];
    load_weights(I.p, W);
    load_weights_bwd(I.p, WB);
    __syncthreads();
    const int wid = wave_id(), lane = lane_id(), li = lane & 15, kq = lane >> 4;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    f32x4 gW2[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) gW2[m][t] = kZero4;
    float gb2[4] = {0.f, 0.f, 0.f, 0.f}, gu[4] = {0.f, 0.f, 0.f, 0.f}, gc0 = 0.f;
    double sq = 0.0;
    const int64_t tiles = (I.n + 15) / 16;
    for (int64_t tt = wave; tt < tiles; tt += static_cast<int64_t>(gridDim.x) * kWavesPerBlock) {
        const int64_t row0 = tt * 16;
        f32x4 y[4];
        float h[4][4], h2[4][4], dO[4], dy[4][4];
        tile_bwd_top(I, W, M, zt, row0, li, kq, Hs[wid], Ds[wid], y, h, h2, dO, dy, &sq);
        bf16x4 bdy[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            bdy[t] = pack4(dy[t][0], dy[t][1], dy[t][2], dy[t][3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gb2[t] += dy[t][q];
                gu[t] += dO[q] * h2[t][q];
            }
        }
        if (li == 0) gc0 += dO[0] + dO[1] + dO[2] + dO[3];
        // [H1 | M]^T dY2: A = H1^T per 16-unit block (D layout of layer 1), then M^T
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const bf16x4 a = pack4(h[m][0], h[m][1], h[m][2], h[m][3]);
#pragma unroll
            for (int t = 0; t < 4; ++t) gW2[m][t] = mfma16(a, bdy[t], gW2[m][t]);
        }
        bf16x4 am;
#pragma unroll
        for (int q = 0; q < 4; ++q) am[q] = static_cast<short>(M[min(row0 + 4 * kq + q, I.n - 1) * kMsg + li]);
#pragma unroll
        for (int t = 0; t < 4; ++t) gW2[4][t] = mfma16(am, bdy[t], gW2[4][t]);
        // dM = dY2 W2[64:80]^T: A = dY2 from Ds, B[k = unit][n = j] = W2[64 + j][unit]
        f32x4 dm = kZero4;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            dm = mfma16(lds4(&Ds[wid][li][16 * ks + 4 * kq]), lds4(&WB.w2r[kH + li][16 * ks + 4 * kq]), dm);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t r = row0 + 4 * kq + q;
            if (r < I.n) dM[r * kMsg + li] = dm[q];
        }
        wave_sync_lds();
    }
    float* pw = part + wave * kPart2;
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) pw[(16 * m + 4 * kq + q) * kH + 16 * t + li] = gW2[m][t][q];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gb2[t] += __shfl_xor(gb2[t], 16, 64);
        gb2[t] += __shfl_xor(gb2[t], 32, 64);
        gu[t] += __shfl_xor(gu[t], 16, 64);
        gu[t] += __shfl_xor(gu[t], 32, 64);
        if (kq == 0) {
            pw[kK2 * kH + 16 * t + li] = gb2[t];
            pw[kK2 * kH + kH + 16 * t + li] = gu[t];
        }
    }
    gc0 += __shfl_xor(gc0, 16, 64);
    gc0 += __shfl_xor(gc0, 32, 64);
    sq += __shfl_xor(sq, 16, 64);
    sq += __shfl_xor(sq, 32, 64);
    if (lane == 0) {
        pw[kK2 * kH + 2 * kH] = gc0;
        loss_part[wave] = sq;
    }
}

// Layer 1's gradients: dH1 = dY2 W2[0:64]^T + dP Wp^T, dY1 = dH1 [y > 0];
// X0^T dY1, sums of dY1, H1^T dP.
__global__ __launch_bounds__(kBlock) void k_net_bwd1(NetIn I, const uint16_t* __restrict__ M,
                                                     const double* __restrict__ zt, const float* __restrict__ dP,
                                                     float* __restrict__ part) {
    __shared__ NetW W;
    __shared__ NetWB WB;
    __shared__ uint16_t Hs[kWavesPerBlock][16][kHS];
    __shared__ uint16_t Ds[kWavesPerBlock][16][kHS];
    load_weights(I.p, W);
    load_weights_bwd(I.p, WB);
    __syncthreads();
    const int wid = wave_id(), lane = lane_id(), li = lane & 15, kq = lane >> 4;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    f32x4 gW1[4], gWp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) gW1[t] = gWp[t] = kZero4;
    float gb1[4] = {0.f, 0.f, 0.f, 0.f};
    double sq = 0.0;
    const int64_t tiles = (I.n + 15) / 16;
    for (int64_t tt = wave; tt < tiles; tt += static_cast<int64_t>(gridDim.x) * kWavesPerBlock) {
        const int64_t row0 = tt * 16;
        f32x4 y[4];
        float h[4][4], h2[4][4], dO[4], dy[4][4];
        tile_bwd_top(I, W, M, zt, row0, li, kq, Hs[wid], Ds[wid], y, h, h2, dO, dy, &sq);
        // dH1: A = dY2 (Ds) with B[k = c][n = m] = W2[m][c]; then A = dP with B[k = j][n = m] = Wp[m][j]
        f32x4 dh[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) dh[t] = kZero4;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x4 a = lds4(&Ds[wid][li][16 * ks + 4 * kq]);
#pragma unroll
            for (int t = 0; t < 4; ++t) dh[t] = mfma16(a, lds4(&WB.w2r[16 * t + li][16 * ks + 4 * kq]), dh[t]);
        }
        const int64_t r = min(row0 + li, I.n - 1);
        const float* pr = dP + r * kMsg + 4 * kq;
        const bf16x4 adp = pack4(pr[0], pr[1], pr[2], pr[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) dh[t] = mfma16(adp, lds4(&WB.wpr[16 * t + li][4 * kq]), dh[t]);
        // dY1 (D layout), zero beyond n
        float dy1[4][4];
        bool live[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) live[q] = row0 + 4 * kq + q < I.n;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                dy1[t][q] = live[q] && y[t][q] > 0.f ? dh[t][q] : 0.f;
                gb1[t] += dy1[t][q];
            }
        // X0^T dY1: A[m = feature li][k = row 4kq+q] (features 8..15 are zero)
        float xf[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float f[8];
            features8(I, min(row0 + 4 * kq + q, I.n - 1), f);
            float v = 0.f;
#pragma unroll
            for (int c = 0; c < 8; ++c) v = li == c ? f[c] : v;
            xf[q] = v;
        }
        const bf16x4 ax = pack4(xf[0], xf[1], xf[2], xf[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) gW1[t] = mfma16(ax, pack4(dy1[t][0], dy1[t][1], dy1[t][2], dy1[t][3]), gW1[t]);
        // H1^T dP: B[k = row 4kq+q][n = j = li]
        float dpq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dpq[q] = live[q] ? dP[(row0 + 4 * kq + q) * kMsg + li] : 0.f;
        const bf16x4 bdp = pack4(dpq[0], dpq[1], dpq[2], dpq[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) gWp[m] = mfma16(pack4(h[m][0], h[m][1], h[m][2], h[m][3]), bdp, gWp[m]);
        wave_sync_lds();
    }
    float* pw = part + wave * kPart1;
    if (kq < 2)  // rows 4kq+q < 8 of X0^T dY1 are the parameters of W1
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) pw[(4 * kq + q) * kH + 16 * t + li] = gW1[t][q];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gb1[t] += __shfl_xor(gb1[t], 16, 64);
        gb1[t] += __shfl_xor(gb1[t], 32, 64);
        if (kq == 0) pw[kF * kH + 16 * t + li] = gb1[t];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) pw[kF * kH + kH + (16 * m + 4 * kq + q) * kMsg + li] = gWp[m][q];
}

// grad[o] = sum over waves, in wave order, of the partials; loss = sum of
// squared errors / n
__global__ void k_net_grad_final(int waves, int64_t n, const float* __restrict__ part1,
                                 const float* __restrict__ part2, const double* __restrict__ loss_part, float* grad,
                                 float* loss) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < kNParams) {
        float t = 0.f;
        if (o < kOffW2)
            for (int w = 0; w < waves; ++w) t += part1[static_cast<int64_t>(w) * kPart1 + o];
        else
            for (int w = 0; w < waves; ++w) t += part2[static_cast<int64_t>(w) * kPart2 + (o - kOffW2)];
        grad[o] = t;
    }
    if (o == 0 && loss) {
        double t = 0.0;
        for (int w = 0; w < waves; ++w) t += loss_part[w];
        *loss = static_cast<float>(t / static_cast<double>(n));
    }
}

// ------------------------------------------------------- weights and Adam
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
    const int wid = wave_id(), lane = lane_id();
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
    const int wid = wave_id(), lane = lane_id();
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
    double* stats_part; double* stats; float* rs; float* s32; float* invd; float* cpart;
    uint16_t* P; uint16_t* M;
    float* dM; float* dP; float* part1; float* part2; double* loss_part; float* grad;
};

constexpr int kStatBlocks = 256;

NetLayout carve_net(Carver& cv, const fj_graph* g, bool training) {
    NetLayout L{};
    const int64_t n = g->n;
    L.stats_part = cv.take<double>(3 * kStatBlocks);
    L.stats = cv.take<double>(4);
    L.rs = cv.take<float>(n);
    L.s32 = cv.take<float>(n);
    L.invd = cv.take<float>(n);
    L.cpart = cv.take<float>((g->tiles_a.nchunks + 1) * kMsg);
    L.P = cv.take<uint16_t>(n * kMsg);
    L.M = cv.take<uint16_t>(n * kMsg);
    if (training) {
        const int64_t waves = static_cast<int64_t>(bwd_blocks(n)) * kWavesPerBlock;
        L.dM = cv.take<float>(n * kMsg);
        L.dP = cv.take<float>(n * kMsg);
        L.part1 = cv.take<float>(waves * kPart1);
        L.part2 = cv.take<float>(waves * kPart2);
        L.loss_part = cv.take<double>(waves);
        L.grad = cv.take<float>(kNParams + 3);
    }
    return L;
}

// the forward up to the message M = nbr(P); then z0 unless training.  ev:
// NULL, or five events recorded before the statistics of s, then after the
// gather of s, after layer 1, after the gather of P and after layer 2.
fj_status net_forward(const fj_graph* g, const double* s, const float* params, double* z0, const NetLayout& L,
                      bool training, hipStream_t st, hipEvent_t* ev = nullptr) {
    const int64_t n = g->n;
    const int bs = 256;
    if (ev) FJ_HIP(hipEventRecord(ev[0], st));
    hipLaunchKernelGGL(k_s_prep, dim3(kStatBlocks), dim3(256), 0, st, n, s, g->opd, L.stats_part, L.s32, L.invd);
    hipLaunchKernelGGL(k_s_final, dim3(1), dim3(64), 0, st, kStatBlocks, n, L.stats_part, L.stats);
    const TileView ta = tile_view_all(g->tiles_a);
    // layer 1's message: the neighbour sum of s over CSR(A)
    if (ta.ntiles > 0)
        hipLaunchKernelGGL(k_nbr_tiles, dim3(waves_to_blocks(ta.ntiles)), dim3(kBlock), 0, st, ta, g->row_ptr, g->col,
                           g->w, L.s32, L.rs);
    if (ta.h1 > ta.h0) {
        hipLaunchKernelGGL(k_nbr_chunks, dim3(waves_to_blocks(ta.nchunks)), dim3(kBlock), 0, st, ta, g->col, g->w,
                           L.s32, L.cpart);
        hipLaunchKernelGGL(k_nbr_combine, dim3(waves_to_blocks(ta.h1 - ta.h0)), dim3(kBlock), 0, st, ta, L.cpart,
                           L.rs);
    }
    const NetIn I{n, s, L.rs, g->opd, L.stats, params, 0.0};
    if (ev) FJ_HIP(hipEventRecord(ev[1], st));
    hipLaunchKernelGGL(k_net_l1, dim3(fwd_blocks(n, 1792)), dim3(kBlock), 0, st, I, L.P);
    if (ev) FJ_HIP(hipEventRecord(ev[2], st));
    // layer 2's message
    hipLaunchKernelGGL(k_agg_rows16, dim3(stride_blocks(g1d(n, 8))), dim3(kBlock), 0, st, n, g->row_ptr, g->col,
                       g->w, L.invd, L.P, L.M);
    if (ta.h1 > ta.h0) {
        hipLaunchKernelGGL(k_agg16_chunks, dim3(waves_to_blocks(ta.nchunks)), dim3(kBlock), 0, st, ta, g->col, g->w,
                           L.P, L.cpart);
        hipLaunchKernelGGL(k_agg16_combine, dim3(waves_to_blocks(ta.h1 - ta.h0)), dim3(kBlock), 0, st, ta, L.cpart,
                           L.invd, L.M);
    }
    if (ev) FJ_HIP(hipEventRecord(ev[3], st));
    if (!training) hipLaunchKernelGGL(k_net_l2, dim3(fwd_blocks(n, 768)), dim3(kBlock), 0, st, I, L.M, z0);
    if (ev) FJ_HIP(hipEventRecord(ev[4], st));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "warm-start forward");
    return FJ_OK;
}

fj_status net_grad(const fj_graph* g, const double* s, const double* zt, const float* params, double rel_floor,
                   const NetLayout& L, float* grad, float* loss, hipStream_t st) {
    const int64_t n = g->n;
    fj_status rc = net_forward(g, s, params, nullptr, L, true, st);
    if (rc) return rc;
    const NetIn I{n, s, L.rs, g->opd, L.stats, params, rel_floor};
    const unsigned nb = bwd_blocks(n);
    hipLaunchKernelGGL(k_net_bwd2, dim3(nb), dim3(kBlock), 0, st, I, L.M, zt, L.dM, L.part2, L.loss_part);
    // dP = nbr^T(dM) over CSR(A^T)
    hipLaunchKernelGGL(k_aggT16_light, dim3(g1d(n * kMsg, kBlock)), dim3(kBlock), 0, st, n, g->t_row_ptr, g->t_col,
                       g->t_w, L.invd, L.dM, L.dP);
    const TileView tt = tile_view_all(g->tiles_t);
    if (tt.h1 > tt.h0)
        hipLaunchKernelGGL(k_aggT16_heavy, dim3(tt.h1 - tt.h0), dim3(1024), 0, st, tt, g->t_row_ptr, g->t_col,
                           g->t_w, L.invd, L.dM, L.dP);
    hipLaunchKernelGGL(k_net_bwd1, dim3(nb), dim3(kBlock), 0, st, I, L.M, zt, L.dP, L.part1);
    hipLaunchKernelGGL(k_net_grad_final, dim3(g1d(kNParams, 256)), dim3(256), 0, st,
                       static_cast<int>(nb * kWavesPerBlock), n, L.part1, L.part2, L.loss_part, grad, loss);
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

extern "C" fj_status fj_wsnet_forward_timed(const fj_graph* g, const double* s, const float* params, double* z0,
                                            void* ws, size_t ws_bytes, double* stage_ms, void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, false);
    if (rc) return rc;
    if (!z0 || !stage_ms) {
        set_error("fj_wsnet_forward_timed: z0 or stage_ms is NULL");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t ev[5] = {};
    int made = 0;
    for (; made < 5; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) break;
    if (made == 5) {
        Carver cv(ws);
        NetLayout L = carve_net(cv, g, false);
        rc = net_forward(g, s, params, z0, L, false, st, ev);
        if (rc == FJ_OK && hipEventSynchronize(ev[4]) != hipSuccess) rc = hip_fail(hipGetLastError(), "event");
        for (int q = 0; q < 4 && rc == FJ_OK; ++q) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
            stage_ms[q] = ms;
        }
    } else {
        rc = hip_fail(hipGetLastError(), "hipEventCreate");
    }
    for (int q = 0; q < made; ++q) (void)hipEventDestroy(ev[q]);
    return rc;
}

extern "C" fj_status fj_wsnet_grad(const fj_graph* g, const double* s, const double* z_target, const float* params,
                                   double rel_floor, float* grad, float* loss, void* ws, size_t ws_bytes,
                                   void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, true);
    if (rc) return rc;
    if (!z_target || !grad || !loss || !std::isfinite(rel_floor)) {
        set_error("fj_wsnet_grad: null argument or non-finite rel_floor");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    NetLayout L = carve_net(cv, g, true);
    return net_grad(g, s, z_target, params, rel_floor, L, grad, loss, static_cast<hipStream_t>(stream));
}

extern "C" fj_status fj_wsnet_train_step(const fj_graph* g, const double* s, const double* z_target, float* params,
                                         float* adam_m, float* adam_v, int32_t step, float lr, double rel_floor,
                                         float* loss, void* ws, size_t ws_bytes, void* stream) {
    fj_status rc = net_args_ok(g, s, params, ws, ws_bytes, true);
    if (rc) return rc;
    if (!z_target || !adam_m || !adam_v || !loss || step < 1 || !(lr > 0.f) || !std::isfinite(rel_floor)) {
        set_error("fj_wsnet_train_step: bad argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    NetLayout L = carve_net(cv, g, true);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = net_grad(g, s, z_target, params, rel_floor, L, L.grad, loss, st);
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

