// ImprovedBLISOR on the GPU: shift (Alg. 2), push rounds (Alg. 1/3 with the
// FIFO relaxed to bulk rounds) or colour-ordered over-relaxed sweeps (Thm. 8
// with Eqs. (sor1)-(sor3)), FP64 certificate (Lemma 7), refinement, unshift.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_grid.h"
#include "fj_sor.h"
#include "fj_tile.h"

namespace fj {
namespace {

constexpr int kMaxRounds = 1 << 20;

inline unsigned grid1d(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }
inline unsigned tile_blocks(int64_t rows) { return static_cast<unsigned>((rows + kBlock - 1) / kBlock); }

// ------------------------------------------------------------------- init
// Alg. 2: s' = s + c, h = eps' s', zhat' = 0, r = s'.  The FP32 threshold is
// rounded down so that |r| <= h32 implies |r| <= h in FP64.
template <typename T>
__global__ void k_init_cold(int64_t n, const double* __restrict__ s, double c, double epsp, T* r, T* h,
                            double* zh, int* bad) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double si = s[i];
    if (!(si >= 0.0) || !isfinite(si)) flag_set(bad);
    double sp = si + c;
    r[i] = static_cast<T>(sp);
    double hv = epsp * sp;
    if constexpr (sizeof(T) == 4) h[i] = __double2float_rd(hv); else h[i] = hv;
    zh[i] = 0.0;
}

// warm start (any zhat' is a valid start, Lemma 4): zhat' = z0 + c
template <typename T>
__global__ void k_init_warm(int64_t n, const double* __restrict__ s, const double* __restrict__ z0, double c,
                            double epsp, T* h, double* zh, int* bad) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double si = s[i], zi = z0[i];
    if (!(si >= 0.0) || !isfinite(si) || !isfinite(zi)) flag_set(bad);
    double hv = epsp * (si + c);
    if constexpr (sizeof(T) == 4) h[i] = __double2float_rd(hv); else h[i] = hv;
    zh[i] = zi + c;
}

// ------------------------------------------------------------ certificate
// r = s' - (I+L) zhat' in FP64 over CSR(A): r_i = s'_i - (1+d_i) zhat'_i +
// sum_j a_ij zhat'_j.  Per block: max |r_i| / h_i and the count of rows with
// |r_i| > h_i (Alg. 3's stopping test).  r_out != NULL also stores r as the
// new tracked residual, which resets FP32 drift (Lemma 4 holds for any
// zhat').  In FP32 it is rounded away from zero: the FP32 threshold is the
// FP64 one rounded down, so a row that fails the FP64 test (|r| > h) then
// passes the FP32 push test |r32| > h32 however close it lies to h; rounded
// to nearest, a row within half an ulp of h could round onto h32, never be
// pushed, and fail every later certificate.  Light tiles finish their rows
// here; heavy rows leave one partial sum per chunk for k_certify_heavy.
struct RowOut {
    double ratio;
    int viol;
};

template <typename T>
__device__ __forceinline__ RowOut certify_row(int64_t i, double sum, const double* __restrict__ s, double c_res,
                                              double c_thr, double epsp, const double* __restrict__ zh,
                                              const double* __restrict__ opd, T* r_out) {
    double ri = (s[i] + c_res) - opd[i] * zh[i] + sum;
    double ratio = fabs(ri) / (epsp * (s[i] + c_thr));
    RowOut o{ratio, !(ratio <= 1.0) ? 1 : 0};  // NaN counts as a violation
    if (!isfinite(o.ratio)) o.ratio = INFINITY;
    if (r_out) {
        if constexpr (sizeof(T) == 4) r_out[i] = ri >= 0.0 ? __double2float_ru(ri) : __double2float_rd(ri);
        else r_out[i] = ri;
    }
    return o;
}

__device__ __forceinline__ void block_max_count(double mx, int vc, double* part_max, long long* part_viol,
                                                int slot) {
    __shared__ double s_mx[kWavesPerBlock];
    __shared__ long long s_vi[kWavesPerBlock];
    const int wid = wave_id();
    mx = wave_max(mx);
    long long v = __popcll(__ballot(vc != 0));
    if (lane_id() == 0) { s_mx[wid] = mx; s_vi[wid] = v; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0; long long c = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) { m = fmax(m, s_mx[k]); c += s_vi[k]; }
        part_max[slot] = m;
        part_viol[slot] = c;
    }
}

// MEAS: the same gathers also form the disagreement D of Table 1 over every
// stored arc, a_ij (zh_i - zh_j)^2 per lane in its arcs' fixed order and a
// fixed-order block sum into part_d[block] (the shift of zh cancels in the
// difference).
template <typename T, bool MEAS = false>
__global__ __launch_bounds__(kBlock) void k_certify_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const float* __restrict__ w, const double* __restrict__ s,
                                                          double c_res, double c_thr, double epsp,
                                                          const double* __restrict__ zh,
                                                          const double* __restrict__ opd, T* r_out,
                                                          double* partial, double* part_max, long long* part_viol,
                                                          double* part_d) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    __shared__ double s_z[MEAS ? kWavesPerBlock : 1][64];
    __shared__ double s_red[kWavesPerBlock];
    const int wid = wave_id(), lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    auto arc = [&](int k) {
        double a = w ? static_cast<double>(w[k]) : 1.0;
        return a * zh[col[k]];
    };
    double dacc = 0.0;
    RowOut ro{0.0, 0};
    if (wv < tv.nchunks) {
        int64_t cidx = tv.c0 + wv;
        int32_t row = tv.heavy_row[tv.chunk_heavy[cidx]];
        int beg = tv.chunk_beg[cidx];
        int end = min(beg + kArcBudget, row_ptr[row + 1]);
        double sum;
        if constexpr (MEAS) {
            const double zi = zh[row];
            sum = chunk_sum(beg, end, [&](int k) {
                const double a = w ? static_cast<double>(w[k]) : 1.0;
                const double zj = zh[col[k]], d = zi - zj;
                dacc += a * d * d;
                return a * zj;
            });
        } else {
            sum = chunk_sum(beg, end, arc);
        }
        if (lane == 0) partial[cidx] = sum;
    } else if (wv - tv.nchunks < tv.ntiles) {
        int64_t tix = tv.t0 + (wv - tv.nchunks);
        if (tv.tile_heavy[tix] < 0) {
            int32_t r0 = tv.tile_start[tix];
            int nrows = tv.tile_start[tix + 1] - r0;
            double sum;
            if constexpr (MEAS) {
                if (lane < nrows) s_z[wid][lane] = zh[r0 + lane];
                wave_sync_lds();
                sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], [&](int k, int slot) {
                    const double a = w ? static_cast<double>(w[k]) : 1.0;
                    const double zj = zh[col[k]], d = s_z[wid][slot] - zj;
                    dacc += a * d * d;
                    return a * zj;
                });
            } else {
                sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], arc);
            }
            if (lane < nrows) ro = certify_row<T>(r0 + lane, sum, s, c_res, c_thr, epsp, zh, opd, r_out);
        }
    }
    block_max_count(ro.ratio, ro.viol, part_max, part_viol, blockIdx.x);
    if constexpr (MEAS) {
        const double t = block_sum<kBlock>(dacc, s_red);
        if (threadIdx.x == 0) part_d[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_certify_heavy(TileView tv, const double* __restrict__ s, double c_res,
                                                          double c_thr, double epsp, const double* __restrict__ zh,
                                                          const double* __restrict__ opd, T* r_out,
                                                          const double* __restrict__ partial, double* part_max,
                                                          long long* part_viol, int slot0) {
    const int wid = wave_id(), lane = lane_id();
    int64_t h = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    RowOut ro{0.0, 0};
    if (h < tv.h1) {
        int32_t c0 = tv.heavy_chunk0[h], c1 = tv.heavy_chunk0[h + 1];
        double sum = 0.0;
        for (int32_t c = c0 + lane; c < c1; c += 64) sum += partial[c];
        sum = wave_sum(sum);
        if (lane == 0) ro = certify_row<T>(tv.heavy_row[h], sum, s, c_res, c_thr, epsp, zh, opd, r_out);
    }
    block_max_count(ro.ratio, ro.viol, part_max, part_viol, slot0 + blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_certify_final(const double* part_max, const long long* part_viol, int64_t nb,
                                                        double* out_max, long long* out_viol) {
    __shared__ double sm[16];
    __shared__ long long sv[16];
    // eight loads of each array in flight per thread (max and count do not
    // depend on the order)
    double m = 0.0; long long v = 0;
    int64_t i = threadIdx.x;
    for (; i + 7 * 1024 < nb; i += 8 * 1024) {
        double pm[8];
        long long pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            pm[u] = part_max[i + u * 1024];
            pv[u] = part_viol[i + u * 1024];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) { m = fmax(m, pm[u]); v += pv[u]; }
    }
    for (; i < nb; i += 1024) { m = fmax(m, part_max[i]); v += part_viol[i]; }
    m = wave_max(m);
    v = wave_sum_ll(v);
    if (lane_id() == 0) { sm[threadIdx.x >> 6] = m; sv[threadIdx.x >> 6] = v; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 16; ++k) { m = fmax(sm[0], sm[k]); sm[0] = m; sv[0] += sv[k]; }
        *out_max = sm[0];
        *out_viol = sv[0];
    }
}

// ---------------------------------------------------------------- push round
// One bulk round of pushes (Alg. 1 / Alg. 3 with the FIFO order relaxed: the
// nodes above threshold at the start of the round are pushed concurrently).
// Lemma 4 holds for any pushed amount, so concurrent pushes keep the invariant;
// with omega = 1 the residual stays >= 0 from a cold start.
//
// A wave owns one tile of CSR(A^T) rows.  Active nodes (|r_v| > h_v) take their
// residual with an atomic exchange, add omega x / (1+d_v) to zhat'_v
// (Eq. (sor1)), leave (1-omega) x at v (Eq. (sor2)), and scatter
// a_uv omega x / (1+d_v) to every u in row v of CSR(A^T) (Eq. (sor3)) with
// hardware float atomics.  The arcs of the active nodes are compacted with a
// ballot + mbcnt prefix into LDS and streamed 64 at a time (merge-path split).
// A heavy node only takes its residual here and publishes the scatter
// coefficient; k_push_heavy scatters its arcs in chunks after this launch.
template <typename T>
__device__ __forceinline__ T take_residual(int64_t v, T* r, const T* __restrict__ inv,
                                           const double* __restrict__ inv64, double* zh, double omega) {
    T x = atomic_exch(&r[v], static_cast<T>(0));
    if (omega != 1.0) atomic_add_noret(&r[v], static_cast<T>((1.0 - omega) * static_cast<double>(x)));
    zh[v] += omega * static_cast<double>(x) * inv64[v];
    return static_cast<T>(omega) * x * inv[v];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_push_light(TileView tv, const int32_t* __restrict__ t_row_ptr,
                                                       const int32_t* __restrict__ t_col,
                                                       const float* __restrict__ t_w, T* r, const T* __restrict__ h,
                                                       const T* __restrict__ inv, const double* __restrict__ inv64,
                                                       double* zh, double omega, T* heavy_coef,
                                                       const int* __restrict__ prev_active, int* this_active,
                                                       unsigned long long* stats) {
    __shared__ int s_beg[kWavesPerBlock][64];
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ T s_cf[kWavesPerBlock][64];
    if (__atomic_load_n(prev_active, __ATOMIC_RELAXED) == 0) return;  // previous round changed nothing
    const int wid = wave_id(), lane = lane_id();
    const int64_t tix = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (tix >= tv.ntiles) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    const int32_t hv = tv.tile_heavy[tix];
    if (hv >= 0) {  // one heavy node: take and publish; the arcs go to k_push_heavy
        if (lane == 0) {
            T cf = 0;
            if (fabs(r[r0]) > h[r0]) {
                cf = take_residual<T>(r0, r, inv, inv64, zh, omega);
                flag_set(this_active);
                stripe_add(stats, 0, 1ull);
                stripe_add(stats, 1, static_cast<unsigned long long>(t_row_ptr[r0 + 1] - t_row_ptr[r0]));
            }
            heavy_coef[hv] = cf;
        }
        return;
    }
    const int64_t v = r0 + lane;
    bool act = false;
    if (lane < nrows) act = fabs(r[v]) > h[v];
    const uint64_t m = __ballot(act);
    if (m == 0) return;
    int beg = 0, deg = 0;
    T cf = 0;
    if (act) {
        cf = take_residual<T>(v, r, inv, inv64, zh, omega);
        beg = t_row_ptr[v];
        deg = t_row_ptr[v + 1] - beg;
    }
    const int slot = lanes_below(m);
    const int cnt = __popcll(m);
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, 63, 64);
    if (act) {
        s_beg[wid][slot] = beg;
        s_pre[wid][slot] = incl - deg;
        s_cf[wid][slot] = cf;
    }
    wave_sync_lds();
    for (int e = lane; e < total; e += 64) {
        int k = tile_find(s_pre[wid], cnt, e);
        int idx = s_beg[wid][k] + (e - s_pre[wid][k]);
        int u = t_col[idx];
        T a = t_w ? static_cast<T>(t_w[idx]) : static_cast<T>(1);
        atomic_add_noret(&r[u], a * s_cf[wid][k]);
    }
    if (lane == 0) {
        flag_set(this_active);
        stripe_add(stats, 0, static_cast<unsigned long long>(cnt));
        stripe_add(stats, 1, static_cast<unsigned long long>(total));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_push_heavy(TileView tv, const int32_t* __restrict__ t_row_ptr,
                                                       const int32_t* __restrict__ t_col,
                                                       const float* __restrict__ t_w, T* r,
                                                       const T* __restrict__ heavy_coef,
                                                       const int* __restrict__ prev_active) {
    if (__atomic_load_n(prev_active, __ATOMIC_RELAXED) == 0) return;
    const int wid = wave_id();
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (c >= tv.nchunks) return;
    const int32_t hv = tv.chunk_heavy[c];
    const T cf = heavy_coef[hv];
    if (cf == static_cast<T>(0)) return;
    const int32_t row = tv.heavy_row[hv];
    const int beg = tv.chunk_beg[c];
    const int end = min(beg + kArcBudget, t_row_ptr[row + 1]);
    for (int k = beg + lane_id(); k < end; k += 64) {
        int u = t_col[k];
        T a = t_w ? static_cast<T>(t_w[k]) : static_cast<T>(1);
        atomic_add_noret(&r[u], a * cf);
    }
}

// ------------------------------------------------------- frontier push rounds
// Alg. 1's queue made concurrent: a round pops every node of the current
// frontier (the round set S^(i) of the proof of Thm. 5), pushes those above
// threshold, and the pushes append the nodes they lift above threshold to the
// next frontier.  Queues are grid-wide arrays of node ids in two degree
// buckets (scatter rows of CSR(A^T) of at most kBigPush arcs: a wave takes 64
// queue entries and scatters their arcs together, merge-path balanced;
// longer: a block per node).  Appends are compacted per wave by ballot and
// prefix count, one global atomic per bucket per wave step.  inq[v] = 1 while
// v is queued.  Ordering without fences (a device-scope fence writes back and
// invalidates the L2 of every XCD on this part): every access here is an
// atomic performed at the device's coherence point, and each one that must
// follow another is issued only after the other has returned.  A popped node
// clears inq, and its read of r depends on the value the clear returned; a
// push that lifts r_u above h_u tests inq[u] only after its add returned.  So
// if the add came after the pop's take, the test sees the cleared flag and
// queues u again; if before, the take collected it.  A node already queued is
// not queued twice.  With omega < 1 a node whose remaining (1 - omega) r is
// still above threshold queues itself.
constexpr int kBigPush = 2048;
constexpr int kFrontierUnroll = 4;
// below this fraction of the nodes pushing per round, rounds pop a frontier queue
constexpr double kFrontierDensity = 0.02;

struct FrontierArgs {
    int32_t* cur[2];   // this round's queues (bucket 0: small, 1: big)
    int32_t* nxt[2];   // the next round's
    const int* cnt_cur;  // [2]
    int* cnt_nxt;        // [2]
    int* inq;
};

__device__ __forceinline__ int push_bucket(const int32_t* __restrict__ t_row_ptr, int u) {
    return t_row_ptr[u + 1] - t_row_ptr[u] > kBigPush ? 1 : 0;
}

// wave-uniform: lanes with `want` append u to the next queue of their bucket
__device__ __forceinline__ void wave_append(bool want, int u, int bucket, const FrontierArgs& F) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const uint64_t m = __ballot(want && bucket == b);
        if (!m) continue;
        int base = 0;
        if (lane_id() == 0) base = atomicAdd(&F.cnt_nxt[b], __popcll(m));
        base = __shfl(base, 0, 64);
        if (want && bucket == b) F.nxt[b][base + lanes_below(m)] = u;
    }
}

// one arc of a push: r_u += delta; a lift above threshold queues u
template <typename T>
__device__ __forceinline__ bool push_arc(int u, T delta, T* r, const T* __restrict__ h, const FrontierArgs& F) {
    const T old = unsafeAtomicAdd(&r[u], delta);
    const T hu = h[u];
    if (!(fabs(old + delta) > hu) || fabs(old) > hu) return false;  // the test waits for the add's return
    return atomicExch(&F.inq[u], 1) == 0;
}

// pop v: clear inq, then take its residual if above threshold; returns the
// push coefficient omega x / (1 + d_v) (0 when v is below threshold) and
// whether v must queue itself again
template <typename T>
__device__ __forceinline__ T pop_node(int v, T* r, const T* __restrict__ h, const T* __restrict__ inv,
                                      const double* __restrict__ inv64, double* zh, double omega,
                                      const FrontierArgs& F, bool* requeue) {
    const int was = atomicExch(&F.inq[v], 0);
    // a zero that the compiler cannot fold, computed from the returned flag:
    // the read of r below is issued only after the clear has returned
    int dep;
    __asm__ volatile("v_mov_b32 %0, 0 ; after %1" : "=v"(dep) : "v"(was));
    T* rv = r + v + dep;
    *requeue = false;
    const T hv = h[v];
    if (!(fabs(unsafeAtomicAdd(rv, static_cast<T>(0))) > hv)) return static_cast<T>(0);  // atomic read
    const T x = atomic_exch(rv, static_cast<T>(0));
    if (omega != 1.0) {
        const T rest = static_cast<T>((1.0 - omega) * static_cast<double>(x));
        const T old = unsafeAtomicAdd(&r[v], rest);
        if (fabs(old + rest) > hv && !(fabs(old) > hv)) *requeue = atomicExch(&F.inq[v], 1) == 0;
    }
    zh[v] += omega * static_cast<double>(x) * inv64[v];
    return static_cast<T>(omega) * x * inv[v];
}

// small bucket: a wave per 64 queue entries, grid-stride
template <typename T>
__global__ __launch_bounds__(kBlock) void k_frontier_small(FrontierArgs F, const int32_t* __restrict__ t_row_ptr,
                                                           const int32_t* __restrict__ t_col,
                                                           const float* __restrict__ t_w, T* r,
                                                           const T* __restrict__ h, const T* __restrict__ inv,
                                                           const double* __restrict__ inv64, double* zh,
                                                           double omega, unsigned long long* stats) {
    __shared__ int s_beg[kWavesPerBlock][64];
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ T s_cf[kWavesPerBlock][64];
    const int cnt = F.cnt_cur[0];
    const int wid = wave_id(), lane = lane_id();
    const int64_t waves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    unsigned long long pushes = 0, visits = 0;
    for (int64_t base = (static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid) * 64; base < cnt;
         base += waves * 64) {
        const int64_t idx = base + lane;
        int v = -1;
        T cf = 0;
        bool requeue = false;
        if (idx < cnt) {
            v = F.cur[0][idx];
            cf = pop_node<T>(v, r, h, inv, inv64, zh, omega, F, &requeue);
        }
        wave_append(requeue, v, 0, F);  // a small node stays small
        const bool act = cf != static_cast<T>(0);
        const uint64_t m = __ballot(act);
        if (m == 0) continue;
        int beg = 0, deg = 0;
        if (act) {
            beg = t_row_ptr[v];
            deg = t_row_ptr[v + 1] - beg;
        }
        const int slot = lanes_below(m);
        const int na = __popcll(m);
        const int incl = wave_incl_scan(deg);
        const int total = __shfl(incl, 63, 64);
        if (act) {
            s_beg[wid][slot] = beg;
            s_pre[wid][slot] = incl - deg;
            s_cf[wid][slot] = cf;
        }
        wave_sync_lds();
        for (int e0 = 0; e0 < total; e0 += 64 * kFrontierUnroll) {  // wave-uniform trip count
            // kFrontierUnroll returning atomics in flight per lane, then their tests
            int u[kFrontierUnroll];
            T delta[kFrontierUnroll], old[kFrontierUnroll];
#pragma unroll
            for (int j = 0; j < kFrontierUnroll; ++j) {
                const int e = e0 + 64 * j + lane;
                u[j] = -1;
                if (e < total) {
                    const int k = tile_find(s_pre[wid], na, e);
                    const int a = s_beg[wid][k] + (e - s_pre[wid][k]);
                    u[j] = t_col[a];
                    delta[j] = (t_w ? static_cast<T>(t_w[a]) : static_cast<T>(1)) * s_cf[wid][k];
                }
            }
#pragma unroll
            for (int j = 0; j < kFrontierUnroll; ++j)
                if (u[j] >= 0) old[j] = unsafeAtomicAdd(&r[u[j]], delta[j]);
#pragma unroll
            for (int j = 0; j < kFrontierUnroll; ++j) {
                bool want = false;
                int bkt = 0;
                if (u[j] >= 0) {
                    const T hu = h[u[j]];
                    if (fabs(old[j] + delta[j]) > hu && !(fabs(old[j]) > hu)) {
                        want = atomicExch(&F.inq[u[j]], 1) == 0;
                        if (want) bkt = push_bucket(t_row_ptr, u[j]);
                    }
                }
                wave_append(want, u[j], bkt, F);
            }
        }
        wave_sync_lds();
        pushes += static_cast<unsigned long long>(na);
        visits += static_cast<unsigned long long>(total);
    }
    if (lane == 0 && pushes) {
        stripe_add(stats, 0, pushes);
        stripe_add(stats, 1, visits);
    }
}

// big bucket: a block per queue entry, grid-stride
template <typename T>
__global__ __launch_bounds__(kBlock) void k_frontier_big(FrontierArgs F, const int32_t* __restrict__ t_row_ptr,
                                                         const int32_t* __restrict__ t_col,
                                                         const float* __restrict__ t_w, T* r,
                                                         const T* __restrict__ h, const T* __restrict__ inv,
                                                         const double* __restrict__ inv64, double* zh, double omega,
                                                         unsigned long long* stats) {
    __shared__ T s_cf;
    __shared__ int s_req;
    const int cnt = F.cnt_cur[1];
    for (int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        const int v = F.cur[1][idx];
        if (threadIdx.x == 0) {
            bool rq = false;
            s_cf = pop_node<T>(v, r, h, inv, inv64, zh, omega, F, &rq);
            s_req = rq ? 1 : 0;
        }
        __syncthreads();
        const T cf = s_cf;
        if (threadIdx.x < 64) wave_append(threadIdx.x == 0 && s_req, v, 1, F);
        if (cf != static_cast<T>(0)) {
            const int beg = t_row_ptr[v], end = t_row_ptr[v + 1];
            for (int k0 = beg; k0 < end; k0 += kBlock) {  // block-uniform trip count
                const int k = k0 + static_cast<int>(threadIdx.x);
                bool want = false;
                int u = 0, bkt = 0;
                if (k < end) {
                    u = t_col[k];
                    const T wgt = t_w ? static_cast<T>(t_w[k]) : static_cast<T>(1);
                    want = push_arc<T>(u, wgt * cf, r, h, F);
                    if (want) bkt = push_bucket(t_row_ptr, u);
                }
                wave_append(want, u, bkt, F);
            }
            if (threadIdx.x == 0) {
                stripe_add(stats, 0, 1ull);
                stripe_add(stats, 1, static_cast<unsigned long long>(end - beg));
            }
        }
        __syncthreads();  // s_cf is rewritten for the next entry
    }
}

// queue every node above threshold (start, or after a refinement re-seeded r)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_frontier_seed(int64_t n, const T* __restrict__ r, const T* __restrict__ h,
                                                          const int32_t* __restrict__ t_row_ptr, FrontierArgs F) {
    const int64_t v = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    bool act = false;
    int bkt = 0;
    if (v < n) {
        act = fabs(r[v]) > h[v];
        F.inq[v] = act ? 1 : 0;
        if (act) bkt = push_bucket(t_row_ptr, static_cast<int>(v));
    }
    wave_append(act, static_cast<int>(v), bkt, F);
}

// end of a round: the consumed counters are cleared for reuse; flag = the
// next frontier is not empty
__global__ void k_frontier_flip(int* cnt_cur, const int* cnt_nxt, int* flag) {
    if (threadIdx.x != 0) return;
    cnt_cur[0] = 0;
    cnt_cur[1] = 0;
    *flag = cnt_nxt[0] + cnt_nxt[1] > 0 ? 1 : 0;
}

// ---------------------------------------------------------- colour-ordered SOR
// Relabelled graph: colour class k occupies a contiguous row range.  Rows of
// one class are not adjacent in A + A^T, so updating them together is exactly
// the sequential Gauss-Seidel update of each (Thm. 8), over-relaxed by omega
// (Eq. (sor1)).  Pull form: r_i = s'_i - (1+d_i) zhat'_i + sum_j a_ij zhat'_j
// is recomputed from the current estimate (equal to the tracked residual by
// Lemma 4), and row i is updated iff |r_i| > h_i = eps' s'_i (Alg. 3's test;
// a margin of 1e-6 h keeps a quiet sweep certified under the FP64 rounding of
// the standalone certificate, which sums in a different order).
// Persistent form of the colour-ordered sweep: one cooperative launch runs up
// to max_sweeps sweeps.  Colour classes are separated by grid barriers (the
// in-kernel equivalent of the per-class launches above).  Rows longer than
// kBigRow are reduced by a whole block, other heavy rows by one wave, light
// tiles by one wave, so no partial sums cross a barrier.  The launch stops
// after the first sweep that updated nothing (all blocks read the same
// per-sweep flag after the sweep's last barrier).
constexpr int kPBlock = 512;
constexpr int kPWaves = kPBlock / 64;

struct SorArgs {
    const int32_t* tile_start;
    const int32_t* tile_heavy;
    const int32_t* heavy_row;
    const int64_t* seg_tile;
    const int64_t* seg_heavy;
    int ncls;
    const int32_t* prow_ptr;
    const int32_t* pcol;
    const float* pw;
    SorState S;
    int max_sweeps;
    int* flags;
    int* bad;
    unsigned long long* stats;
    GridSync gs;
};

__global__ __launch_bounds__(kPBlock) void k_sor_persistent(SorArgs a) {
    __shared__ int s_pre[kPWaves][65];
    __shared__ double s_acc[kPWaves][64];
    __shared__ double s_red[kPWaves];
    const int wid = wave_id(), lane = lane_id();
    const int64_t gw = static_cast<int64_t>(blockIdx.x) * kPWaves + wid;
    const int64_t G = static_cast<int64_t>(gridDim.x) * kPWaves;
    unsigned epoch = 0;
    unsigned long long my_upd = 0;
    auto arc = [&](int k) {
        double w = a.pw ? static_cast<double>(a.pw[k]) : 1.0;
        return w * a.S.zh[a.pcol[k]];
    };
    for (int sw = 0; sw < a.max_sweeps; ++sw) {
        int* upd = a.flags + sw;
        for (int k = 0; k < a.ncls; ++k) {
            const int64_t h0 = a.seg_heavy[k], h1 = a.seg_heavy[k + 1];
            for (int64_t hh = h0 + blockIdx.x; hh < h1; hh += gridDim.x) {
                const int32_t row = a.heavy_row[hh];
                const int b = a.prow_ptr[row], e = a.prow_ptr[row + 1];
                if (e - b <= kBigRow) continue;  // uniform across the block
                double sum = block_arc_sum(b, e, s_red, arc);
                if (threadIdx.x == 0) {
                    bool nf = false;
                    if (sor_row(row, sum, a.S, &nf)) {
                        flag_set(upd);
                        ++my_upd;
                    }
                    if (nf) flag_set(a.bad);
                }
            }
            const int64_t t0 = a.seg_tile[k], t1 = a.seg_tile[k + 1];
            for (int64_t tix = t0 + gw; tix < t1; tix += G) {
                const int32_t r0 = a.tile_start[tix];
                if (a.tile_heavy[tix] >= 0) {
                    const int b = a.prow_ptr[r0], e = a.prow_ptr[r0 + 1];
                    if (e - b > kBigRow) continue;  // done by a block above
                    double sum = chunk_sum(b, e, arc);
                    if (lane == 0) {
                        bool nf = false;
                        if (sor_row(r0, sum, a.S, &nf)) {
                            flag_set(upd);
                            ++my_upd;
                        }
                        if (nf) flag_set(a.bad);
                    }
                } else {
                    const int nrows = a.tile_start[tix + 1] - r0;
                    double sum = tile_row_sums(a.prow_ptr, r0, nrows, s_pre[wid], s_acc[wid], arc);
                    bool u = false, nf = false;
                    if (lane < nrows) u = sor_row(r0 + lane, sum, a.S, &nf);
                    const uint64_t um = __ballot(u);
                    const uint64_t nm = __ballot(nf);
                    if (lane == 0) {
                        if (um) {
                            flag_set(upd);
                            my_upd += __popcll(um);
                        }
                        if (nm) flag_set(a.bad);
                    }
                }
            }
            if (!grid_barrier(a.gs, epoch)) {
                if (lane == 0 && my_upd) stripe_add(a.stats, 0, my_upd);
                return;
            }
        }
        if (__hip_atomic_load(upd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
    }
    if (lane == 0 && my_upd) stripe_add(a.stats, 0, my_upd);
}


__global__ void k_unshift(int64_t n, const double* __restrict__ zh, double c, double* z) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) z[i] = zh[i] - c;
}

// --------------------------------------------------------------- workspace
struct SolveLayout {
    void* r; void* h; double* zh; double* zh2; double* sp; int32_t* zq;
    int* flags; int* one; int* bad; unsigned long long* stats;
    double* partial; void* heavy_coef; unsigned* barrier; int* abort;
    double* part_max; long long* part_viol; double* cert_max; long long* cert_viol;
    unsigned long long* hacc; unsigned long long* zmax_bits; double* zsh; int32_t* zqsh;
    double* ub; double* ub_tail; int* modes; unsigned long long* snaps;
    int32_t* fq[2][2]; int* fcnt; int* inq;  // frontier push: queues [parity][bucket], counters [parity][bucket]
    double* part_d; void* mws;  // opts.measures: D per certificate block; the measures' own workspace
};


int64_t cert_parts(const fj_graph* g) {
    return waves_to_blocks(g->tiles_a.nchunks + g->tiles_a.ntiles) + waves_to_blocks(g->tiles_a.nheavy) + 2;
}

SolveLayout carve_solve(Carver& cv, const fj_graph* g, int precision, bool frontier = false) {
    SolveLayout L{};
    const int64_t n = g->n;
    size_t tsz = precision == FJ_FP64 ? sizeof(double) : sizeof(float);
    L.r = cv.take<char>(tsz * n);
    L.h = cv.take<char>(tsz * n);
    L.zh = cv.take<double>(n);
    L.zh2 = cv.take<double>(n);
    L.sp = cv.take<double>(n);
    L.zq = cv.take<int32_t>(n);
    L.flags = cv.take<int>(kMaxRounds);
    L.one = cv.take<int>(1);
    L.bad = cv.take<int>(1);
    L.barrier = cv.take<unsigned>(1);
    L.abort = cv.take<int>(1);
    L.stats = cv.take<unsigned long long>(kStripes * kStripeStride);
    int64_t nch = std::max(g->tiles_a.nchunks, g->tiles_p.nchunks) + 1;
    L.partial = cv.take<double>(nch);
    L.heavy_coef = cv.take<char>(tsz * (g->tiles_t.nheavy + 1));
    L.hacc = cv.take<unsigned long long>(2 * std::max(g->tiles_p.nheavy, g->tiles_a.nheavy) + 2);
    L.zmax_bits = cv.take<unsigned long long>(1);
    L.zsh = cv.take<double>(n + 1);  // merged tail, or every row in gather-form rounds
    L.zqsh = cv.take<int32_t>(n + 1);
    L.ub = cv.take<double>(n + 1);       // bound skipping: residual bound per row
    L.ub_tail = cv.take<double>(n + 1);  // and the merged tail's collected adds
    L.modes = cv.take<int>(kMaxRounds);
    L.snaps = cv.take<unsigned long long>(kMaxRounds);
    int64_t nb = cert_parts(g);
    L.part_max = cv.take<double>(nb);
    L.part_viol = cv.take<long long>(nb);
    L.cert_max = cv.take<double>(1);
    L.cert_viol = cv.take<long long>(1);
    L.part_d = cv.take<double>(nb);
    L.mws = cv.take<char>(measures_ws_bytes(g));
    if (frontier) {
        for (int par = 0; par < 2; ++par)
            for (int b = 0; b < 2; ++b) L.fq[par][b] = cv.take<int32_t>(n + 1);
        L.fcnt = cv.take<int>(4);
        L.inq = cv.take<int>(n + 1);
    }
    return L;
}

// Optional per-launch timing of the iteration kernels with HIP events.
struct LaunchTimer {
    bool on = false;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    fj_status before() { return on ? record() : FJ_OK; }
    fj_status after() { return on ? record() : FJ_OK; }
    fj_status record() {
        if (used == ev.size()) {
            hipEvent_t e;
            FJ_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        FJ_HIP(hipEventRecord(ev[used++], st));
        return FJ_OK;
    }
    fj_status total_ms(double* ms, int64_t* launches) {
        *ms = 0.0;
        *launches = static_cast<int64_t>(used / 2);
        if (!on || used == 0) return FJ_OK;
        FJ_HIP(hipEventSynchronize(ev[used - 1]));
        for (size_t k = 0; k + 1 < used; k += 2) {
            float t = 0.0f;
            FJ_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            *ms += t;
        }
        return FJ_OK;
    }
    ~LaunchTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

struct HostStats {
    unsigned long long pushes = 0, visits = 0, skipped = 0, skipped_arcs_fix = 0, skipped_arcs_fp64 = 0;
    unsigned long long bound_adds = 0;
    unsigned long long skipped_heavy_fix = 0;  // of skipped_arcs_fix, the arcs of heavy rows
};

fj_status read_stats(const SolveLayout& L, hipStream_t st, HostStats* hs) {
    std::vector<unsigned long long> buf(kStripes * kStripeStride);
    FJ_HIP(hipMemcpyAsync(buf.data(), L.stats, sizeof(unsigned long long) * buf.size(), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    hs->pushes = hs->visits = hs->skipped = hs->skipped_arcs_fix = hs->skipped_arcs_fp64 = hs->bound_adds = 0;
    hs->skipped_heavy_fix = 0;
    for (int k = 0; k < kStripes; ++k) {
        hs->pushes += buf[k * kStripeStride + 0];
        hs->visits += buf[k * kStripeStride + 1];
        hs->skipped += buf[k * kStripeStride + 2];
        hs->skipped_arcs_fix += buf[k * kStripeStride + 3];
        hs->skipped_arcs_fp64 += buf[k * kStripeStride + 4];
        hs->bound_adds += buf[k * kStripeStride + 5];
        hs->skipped_heavy_fix += buf[k * kStripeStride + 6];
    }
    hs->skipped_arcs_fix += hs->skipped_heavy_fix;
    return FJ_OK;
}

// FJ_TRACE (any value but empty or 0) in the environment: one JSON line on
// stderr per host check of a solve (cumulative updates, arcs and skipped
// rows after each batch of rounds or sweeps) and per FP64 certificate.
bool trace_on() {
    static const bool on = [] {
        const char* e = std::getenv("FJ_TRACE");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}
void trace_batch(const char* sched, const char* mode, int64_t rounds, int used, const HostStats& hs) {
    std::fprintf(stderr,
                 "{\"fj_trace\": \"%s\", \"event\": \"batch\", \"mode\": \"%s\", \"rounds\": %lld, "
                 "\"batch_rounds\": %d, \"updates\": %llu, \"edge_visits\": %llu, \"skipped_rows\": %llu}\n",
                 sched, mode, static_cast<long long>(rounds), used, hs.pushes, hs.visits, hs.skipped);
}
void trace_cert(const char* sched, int64_t rounds, double max_ratio, long long viol, int refinements) {
    std::fprintf(stderr,
                 "{\"fj_trace\": \"%s\", \"event\": \"certificate\", \"rounds\": %lld, \"max_ratio\": %.17g, "
                 "\"violations\": %lld, \"refinements\": %d}\n",
                 sched, static_cast<long long>(rounds), max_ratio, viol, refinements);
}

// c_res: shift already inside zh (residual of the shifted system); c_thr: shift
// of the threshold h = eps' (s + c_thr)
// MEAS: the gather pass also leaves D's per-block sums in L.part_d (blocks
// returned in *d_blocks) for measures_with_d.
template <typename T, bool MEAS = false>
fj_status certify(const fj_graph* g, const double* s, double c_res, double c_thr, double epsp, const double* zh,
                  T* r_out, const SolveLayout& L, hipStream_t st, double* max_ratio, long long* viol,
                  int64_t* d_blocks = nullptr) {
    const int64_t n = g->n;
    if (n > 0) {
        TileView tv = tile_view_all(g->tiles_a);
        unsigned nb1 = waves_to_blocks(tv.nchunks + tv.ntiles);
        unsigned nb2 = waves_to_blocks(tv.h1 - tv.h0);
        if (d_blocks) *d_blocks = nb1;
        hipLaunchKernelGGL((k_certify_tiles<T, MEAS>), dim3(nb1), dim3(kBlock), 0, st, tv, g->row_ptr, g->col, g->w, s,
                           c_res, c_thr, epsp, zh, g->opd, r_out, L.partial, L.part_max, L.part_viol, L.part_d);
        if (nb2 > 0)
            hipLaunchKernelGGL(k_certify_heavy<T>, dim3(nb2), dim3(kBlock), 0, st, tv, s, c_res, c_thr, epsp, zh,
                               g->opd, r_out, L.partial, L.part_max, L.part_viol, static_cast<int>(nb1));
        hipLaunchKernelGGL(k_certify_final, dim3(1), dim3(1024), 0, st, L.part_max, L.part_viol,
                           static_cast<int64_t>(nb1 + nb2), L.cert_max, L.cert_viol);
    } else {
        FJ_HIP(hipMemsetAsync(L.cert_max, 0, sizeof(double), st));
        FJ_HIP(hipMemsetAsync(L.cert_viol, 0, sizeof(long long), st));
    }
    FJ_HIP(hipMemcpyAsync(max_ratio, L.cert_max, sizeof(double), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipMemcpyAsync(viol, L.cert_viol, sizeof(long long), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    return FJ_OK;
}

template <typename T>
fj_status solve_push(const fj_graph* g, const double* s, const fj_solve_opts* o, double epsp, double* z,
                     const SolveLayout& L, fj_solve_stats* out, hipStream_t st, int64_t cap) {
    const int64_t n = g->n;
    T* r = static_cast<T*>(L.r);
    T* h = static_cast<T*>(L.h);
    T* coef = static_cast<T*>(L.heavy_coef);
    const T* inv = sizeof(T) == 4 ? reinterpret_cast<const T*>(g->inv32) : reinterpret_cast<const T*>(g->inv64);
    const int bs = 256;
    if (n > 0) {
        if (o->z0) {
            hipLaunchKernelGGL(k_init_warm<T>, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, s, o->z0, o->c, epsp, h, L.zh,
                               L.bad);
            double mr; long long vi;
            fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, r, L, st, &mr, &vi);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(k_init_cold<T>, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, s, o->c, epsp, r, h, L.zh,
                               L.bad);
        }
    }
    int hbad = 0;
    FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("s must be finite and >= 0, and z0 finite");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const int K = o->check_every > 0 ? o->check_every : 8;
    const int max_ref = o->max_refinements >= 0 ? o->max_refinements : 8;
    const TileView tv = tile_view_all(g->tiles_t);
    const unsigned nb_light = waves_to_blocks(tv.ntiles);
    const unsigned nb_heavy = waves_to_blocks(tv.nchunks);
    int64_t rounds = 0, launches = 0;
    int refinements = 0;
    bool converged = false, capped = false;
    double max_ratio = 0.0;
    std::vector<int> hf(K);
    HostStats hs;
    LaunchTimer timer;
    timer.on = o->profile != 0;
    timer.st = st;
    while (true) {
        // rounds until one finds no node above threshold
        bool quiet = false;
        const int* prev = L.one;
        while (!quiet) {
            if (rounds + K > kMaxRounds) { capped = true; break; }
            FJ_HIP(hipMemsetAsync(L.flags + rounds, 0, sizeof(int) * K, st));
            for (int b = 0; b < K; ++b) {
                int* cur = L.flags + rounds + b;
                if (n > 0) {
                    fj_status rc0 = timer.before();
                    if (rc0) return rc0;
                    hipLaunchKernelGGL(k_push_light<T>, dim3(nb_light), dim3(kBlock), 0, st, tv, g->t_row_ptr,
                                       g->t_col, g->t_w, r, h, inv, g->inv64, L.zh, o->omega, coef, prev, cur,
                                       L.stats);
                    ++launches;
                    if (nb_heavy > 0) {
                        hipLaunchKernelGGL(k_push_heavy<T>, dim3(nb_heavy), dim3(kBlock), 0, st, tv, g->t_row_ptr,
                                           g->t_col, g->t_w, r, coef, prev);
                        ++launches;
                    }
                    rc0 = timer.after();
                    if (rc0) return rc0;
                }
                prev = cur;
            }
            FJ_HIP(hipMemcpyAsync(hf.data(), L.flags + rounds, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            fj_status rc = read_stats(L, st, &hs);
            if (rc) return rc;
            int used = K;
            for (int b = 0; b < K; ++b)
                if (hf[b] == 0) { used = b; quiet = true; break; }
            rounds += used;
            if (n == 0) quiet = true;
            if (trace_on()) trace_batch("push", "scan", rounds, used, hs);
            if (static_cast<int64_t>(hs.visits) > cap) { capped = true; break; }
        }
        if (capped) break;
        long long viol = 0;
        fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, r, L, st, &max_ratio, &viol);
        if (rc) return rc;
        if (trace_on()) trace_cert("push", rounds, max_ratio, viol, refinements);
        if (viol == 0) { converged = true; break; }
        if (!std::isfinite(max_ratio) || refinements >= max_ref) break;
        ++refinements;  // r now holds the FP64 residual rounded to T; resume pushing
    }
    if (!converged) {
        long long viol = 0;
        fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, static_cast<T*>(nullptr), L, st, &max_ratio, &viol);
        if (rc) return rc;
    }
    if (n > 0) hipLaunchKernelGGL(k_unshift, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, L.zh, o->c, z);
    FJ_HIP(hipStreamSynchronize(st));
    {
        fj_status rc0 = timer.total_ms(&out->kernel_ms, &out->kernel_launches);
        if (rc0) return rc0;
    }
    out->pushes = static_cast<int64_t>(hs.pushes);
    out->edge_visits = static_cast<int64_t>(hs.visits);
    out->rounds = rounds;
    out->launches = launches;
    out->refinements = refinements;
    out->certified = converged ? 1 : 0;
    out->max_ratio = max_ratio;
    if (!converged) {
        set_error(capped ? "work cap reached before the certificate held"
                         : "certificate failed after the refinement budget (or the iteration diverged)");
        return FJ_ERR_NOT_CONVERGED;
    }
    return FJ_OK;
}

// Push rounds that switch from a scan of every node to a frontier queue
// (push_scatter = 2).  While many nodes are above threshold a round scans
// all of them and scatters with atomics that return nothing (k_push_light /
// k_push_heavy); once a batch of check_every rounds averaged fewer pushes per
// round than kFrontierDensity of the nodes, the queue is seeded with the
// nodes above threshold and each round pops only the previous round's
// appends, whose detection needs atomics that return the old residual.  The
// host checks every check_every rounds; a round with nothing to push (scan)
// or an empty next frontier is quiet.  FP32 or FP64 residual; the order of
// concurrent atomic additions is not fixed, so the pushes (not the
// certificate) may differ run to run.
template <typename T>
fj_status solve_push_frontier(const fj_graph* g, const double* s, const fj_solve_opts* o, double epsp, double* z,
                              const SolveLayout& L, fj_solve_stats* out, hipStream_t st, int64_t cap) {
    const int64_t n = g->n;
    T* r = static_cast<T*>(L.r);
    T* h = static_cast<T*>(L.h);
    const T* inv = sizeof(T) == 4 ? reinterpret_cast<const T*>(g->inv32) : reinterpret_cast<const T*>(g->inv64);
    const int bs = 256;
    if (n > 0) {
        if (o->z0) {
            hipLaunchKernelGGL(k_init_warm<T>, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, s, o->z0, o->c, epsp, h, L.zh,
                               L.bad);
            double mr; long long vi;
            fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, r, L, st, &mr, &vi);
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(k_init_cold<T>, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, s, o->c, epsp, r, h, L.zh,
                               L.bad);
        }
    }
    int hbad = 0;
    FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("s must be finite and >= 0, and z0 finite");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const int K = o->check_every > 0 ? o->check_every : 8;
    const int max_ref = o->max_refinements >= 0 ? o->max_refinements : 8;
    // grids sized to fill the chip; the kernels stride over their queue
    const unsigned nb_small = 2048, nb_big = 512;
    const TileView tv = tile_view_all(g->tiles_t);
    const unsigned nb_light = waves_to_blocks(tv.ntiles);
    const unsigned nb_heavy = waves_to_blocks(tv.nchunks);
    T* coef = static_cast<T*>(L.heavy_coef);
    int64_t rounds = 0, launches = 0;
    int refinements = 0;
    bool converged = false, capped = false;
    double max_ratio = 0.0;
    std::vector<int> hf(K);
    HostStats hs;
    LaunchTimer timer;
    timer.on = o->profile != 0;
    timer.st = st;
    auto args = [&](int par) {
        FrontierArgs F{};
        F.cur[0] = L.fq[par][0];
        F.cur[1] = L.fq[par][1];
        F.nxt[0] = L.fq[par ^ 1][0];
        F.nxt[1] = L.fq[par ^ 1][1];
        F.cnt_cur = L.fcnt + 2 * par;
        F.cnt_nxt = L.fcnt + 2 * (par ^ 1);
        F.inq = L.inq;
        return F;
    };
    int par = 0;
    int64_t frontier_rounds = 0;
    while (true) {
        bool queued = false;  // this phase has switched to the frontier queue
        bool quiet = n == 0;
        const int* prev = L.one;
        while (!quiet) {
            if (rounds + K > kMaxRounds) { capped = true; break; }
            FJ_HIP(hipMemsetAsync(L.flags + rounds, 0, sizeof(int) * K, st));
            const unsigned long long pushes_before = hs.pushes;
            if (!queued) {  // scan rounds
                for (int b = 0; b < K; ++b) {
                    int* cur = L.flags + rounds + b;
                    fj_status rc0 = timer.before();
                    if (rc0) return rc0;
                    hipLaunchKernelGGL(k_push_light<T>, dim3(nb_light), dim3(kBlock), 0, st, tv, g->t_row_ptr,
                                       g->t_col, g->t_w, r, h, inv, g->inv64, L.zh, o->omega, coef, prev, cur,
                                       L.stats);
                    ++launches;
                    if (nb_heavy > 0) {
                        hipLaunchKernelGGL(k_push_heavy<T>, dim3(nb_heavy), dim3(kBlock), 0, st, tv, g->t_row_ptr,
                                           g->t_col, g->t_w, r, coef, prev);
                        ++launches;
                    }
                    rc0 = timer.after();
                    if (rc0) return rc0;
                    prev = cur;
                }
                FJ_HIP(hipMemcpyAsync(hf.data(), L.flags + rounds, sizeof(int) * K, hipMemcpyDeviceToHost, st));
                fj_status rc = read_stats(L, st, &hs);
                if (rc) return rc;
                int used = K;
                for (int b = 0; b < K; ++b)
                    if (hf[b] == 0) { used = b; quiet = true; break; }
                rounds += used;
                if (trace_on()) trace_batch("push", "scan", rounds, used, hs);
                if (static_cast<int64_t>(hs.visits) > cap) { capped = true; break; }
                if (!quiet && static_cast<double>(hs.pushes - pushes_before) <
                                  kFrontierDensity * static_cast<double>(n) * static_cast<double>(used)) {
                    // sparse: the frontier is every node above threshold now
                    FJ_HIP(hipMemsetAsync(L.fcnt, 0, sizeof(int) * 4, st));
                    hipLaunchKernelGGL(k_frontier_seed<T>, dim3(grid1d(n, kBlock)), dim3(kBlock), 0, st, n, r, h,
                                       g->t_row_ptr, args(1));
                    ++launches;
                    par = 0;  // the seed filled the queues of parity 0 (the "next" of parity 1)
                    queued = true;
                }
                continue;
            }
            for (int b = 0; b < K; ++b) {
                const FrontierArgs F = args(par);
                fj_status rc0 = timer.before();
                if (rc0) return rc0;
                hipLaunchKernelGGL(k_frontier_small<T>, dim3(nb_small), dim3(kBlock), 0, st, F, g->t_row_ptr,
                                   g->t_col, g->t_w, r, h, inv, g->inv64, L.zh, o->omega, L.stats);
                hipLaunchKernelGGL(k_frontier_big<T>, dim3(nb_big), dim3(kBlock), 0, st, F, g->t_row_ptr, g->t_col,
                                   g->t_w, r, h, inv, g->inv64, L.zh, o->omega, L.stats);
                rc0 = timer.after();
                if (rc0) return rc0;
                hipLaunchKernelGGL(k_frontier_flip, dim3(1), dim3(64), 0, st, L.fcnt + 2 * par,
                                   L.fcnt + 2 * (par ^ 1), L.flags + rounds + b);
                launches += 3;
                par ^= 1;
            }
            FJ_HIP(hipMemcpyAsync(hf.data(), L.flags + rounds, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            fj_status rc = read_stats(L, st, &hs);
            if (rc) return rc;
            int used = K;
            for (int b = 0; b < K; ++b)
                if (hf[b] == 0) { used = b + 1; quiet = true; break; }
            rounds += used;
            frontier_rounds += used;
            if (trace_on()) trace_batch("push", "queue", rounds, used, hs);
            if (static_cast<int64_t>(hs.visits) > cap) { capped = true; break; }
        }
        if (capped) break;
        long long viol = 0;
        fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, r, L, st, &max_ratio, &viol);
        if (rc) return rc;
        if (trace_on()) trace_cert("push", rounds, max_ratio, viol, refinements);
        if (viol == 0) { converged = true; break; }
        if (!std::isfinite(max_ratio) || refinements >= max_ref) break;
        ++refinements;  // r now holds the FP64 residual rounded to T; the rounds resume from it
    }
    if (!converged) {
        long long viol = 0;
        fj_status rc = certify<T>(g, s, o->c, o->c, epsp, L.zh, static_cast<T*>(nullptr), L, st, &max_ratio, &viol);
        if (rc) return rc;
    }
    if (n > 0) hipLaunchKernelGGL(k_unshift, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, L.zh, o->c, z);
    FJ_HIP(hipStreamSynchronize(st));
    {
        fj_status rc0 = timer.total_ms(&out->kernel_ms, &out->kernel_launches);
        if (rc0) return rc0;
    }
    out->pushes = static_cast<int64_t>(hs.pushes);
    out->edge_visits = static_cast<int64_t>(hs.visits);
    out->rounds = rounds;
    out->launches = launches;
    out->refinements = refinements;
    out->certified = converged ? 1 : 0;
    out->max_ratio = max_ratio;
    out->mirror_rounds = frontier_rounds;  // push rounds: the rounds that popped a frontier queue
    if (!converged) {
        set_error(capped ? "work cap reached before the certificate held"
                         : "certificate failed after the refinement budget (or the iteration diverged)");
        return FJ_ERR_NOT_CONVERGED;
    }
    return FJ_OK;
}

// The 32-bit copy of the SOR kernels holds |zhat'| < 2.  The iterates stay
// within the range of s' and of the start, up to the overshoot of
// over-relaxation, so the copy is used only when that range (the init
// kernel's magnitude bound, as bits) is below 1.5; otherwise every sweep
// gathers FP64.
bool fix_range_ok(unsigned long long zmax_bits) {
    double m;
    std::memcpy(&m, &zmax_bits, sizeof(m));
    return m < 1.5;
}

// Bulk rounds (Alg. 1 / Alg. 3 with the FIFO order relaxed to the round sets
// of the proof of Thm. 5) in gather form: every round recomputes each row's
// residual r_i = s'_i - (1+d_i) zhat'_i + sum_j a_ij zhat'_j from the estimate
// of the round's start (equal to the tracked residual by Lemma 4) and moves
// the rows above threshold by omega r_i / (1+d_i).  That is the same update
// as every active node pushing at once, without the atomic scatter to its
// in-neighbours: one launch of the class sweep over all of CSR(A) with shadow
// writes (so all rows read the round's start), then a commit.
fj_status solve_rounds_gather(const fj_graph* g, const double* s, const fj_solve_opts* o, double epsp, double* z,
                              const SolveLayout& L, fj_solve_stats* out, hipStream_t st, int64_t cap) {
    const int64_t n = g->n;
    const int bs = 256;
    FJ_HIP(hipMemsetAsync(L.hacc, 0, sizeof(unsigned long long) * (2 * g->tiles_a.nheavy + 2), st));
    FJ_HIP(hipMemsetAsync(L.zmax_bits, 0, sizeof(unsigned long long), st));
    if (n > 0)
        hipLaunchKernelGGL(k_sor_init, dim3(std::min<unsigned>(grid1d(n, bs), 2048u)), dim3(bs), 0, st, n,
                           static_cast<const int32_t*>(nullptr), s, o->z0, o->c, L.sp, L.zh, L.zq, L.bad,
                           L.zmax_bits);
    int hbad = 0;
    unsigned long long hzmax = 0;
    FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipMemcpyAsync(&hzmax, L.zmax_bits, sizeof(hzmax), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("s must be finite and >= 0, and z0 finite");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const int K = o->check_every > 0 ? o->check_every : 8;
    const int max_ref = o->max_refinements >= 0 ? o->max_refinements : 8;
    const TileView tv = tile_view_all(g->tiles_a);
    const unsigned grid = waves_to_blocks(tv.nchunks + tv.ntiles);
    SorState S64{L.sp, g->opd, g->inv64, L.zh, L.zq, o->omega, 1.0 - 1e-6, epsp, L.hacc, L.zmax_bits,
                 L.zsh, L.zqsh, 0};
    SorState SMIR = S64;
    SMIR.thr = 0.95;
    bool mirror = o->precision == FJ_FP32 && o->gather_bits != 64 && fix_range_ok(hzmax);
    int64_t rounds = 0, launches = 0, mirror_rounds = 0;
    int refinements = 0;
    bool converged = false, capped = false, diverged = false;
    double max_ratio = 0.0;
    std::vector<int> hf(K);
    LaunchTimer timer;
    timer.on = o->profile != 0;
    timer.st = st;
    while (true) {
        bool quiet = false;
        while (!quiet) {
            if (rounds + K > kMaxRounds || (rounds + K) * (g->nnz + n) > cap) { capped = true; break; }
            FJ_HIP(hipMemsetAsync(L.flags + rounds, 0, sizeof(int) * K, st));
            for (int b = 0; b < K; ++b) {
                int* cur = L.flags + rounds + b;
                const int* prev = b > 0 ? cur - 1 : nullptr;
                if (n == 0) continue;
                fj_status rc0 = timer.before();
                if (rc0) return rc0;
                if (mirror)
                    hipLaunchKernelGGL((k_sor_class<true, true, false>), dim3(grid), dim3(kBlock), 0, st, tv,
                                       g->row_ptr, g->col, g->w, SMIR, prev, cur, L.bad, L.stats, nullptr);
                else
                    hipLaunchKernelGGL((k_sor_class<false, true, false>), dim3(grid), dim3(kBlock), 0, st, tv,
                                       g->row_ptr, g->col, g->w, S64, prev, cur, L.bad, L.stats, nullptr);
                hipLaunchKernelGGL(k_sor_commit, dim3(grid1d(n, bs)), dim3(bs), 0, st, static_cast<int64_t>(0), n,
                                   L.zsh, L.zqsh, L.zh, L.zq, prev);
                launches += 2;
                rc0 = timer.after();
                if (rc0) return rc0;
            }
            FJ_HIP(hipMemcpyAsync(hf.data(), L.flags + rounds, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
            FJ_HIP(hipStreamSynchronize(st));
            if (hbad) { diverged = true; break; }
            int used = K;
            for (int b = 0; b < K; ++b)
                if (hf[b] == 0) { used = b + 1; quiet = true; break; }
            rounds += used;
            if (mirror) mirror_rounds += used;
            if (n == 0) quiet = true;
            if (trace_on()) {
                HostStats hs;
                fj_status rc0 = read_stats(L, st, &hs);
                if (rc0) return rc0;
                trace_batch("push", mirror ? "gather fixed-point" : "gather fp64", rounds, used, hs);
            }
        }
        if (capped || diverged) break;
        long long viol = 0;
        fj_status rc = certify<double>(g, s, o->c, o->c, epsp, L.zh, static_cast<double*>(nullptr), L, st,
                                       &max_ratio, &viol);
        if (rc) return rc;
        if (viol == 0) { converged = true; break; }
        if (mirror) {  // finish with FP64 gathers
            mirror = false;
            continue;
        }
        if (refinements >= max_ref) break;
        ++refinements;
    }
    if (!converged && (capped || diverged)) {
        long long viol = 0;
        fj_status rc = certify<double>(g, s, o->c, o->c, epsp, L.zh, static_cast<double*>(nullptr), L, st,
                                       &max_ratio, &viol);
        if (rc) return rc;
    }
    if (n > 0) hipLaunchKernelGGL(k_unshift, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, L.zh, o->c, z);
    HostStats hs;
    fj_status rc = read_stats(L, st, &hs);
    if (rc) return rc;
    rc = timer.total_ms(&out->kernel_ms, &out->kernel_launches);
    if (rc) return rc;
    out->mirror_rounds = mirror_rounds;
    out->pushes = static_cast<int64_t>(hs.pushes);
    out->edge_visits = rounds * g->nnz;
    out->rounds = rounds;
    out->launches = launches;
    out->refinements = refinements;
    out->certified = converged ? 1 : 0;
    out->max_ratio = max_ratio;
    if (!converged) {
        set_error(diverged ? "rounds diverged (non-finite residual)"
                           : capped ? "work cap reached before the certificate held"
                                    : "certificate failed after the refinement budget");
        return FJ_ERR_NOT_CONVERGED;
    }
    return FJ_OK;
}

// One launch of k_sor_class over tv: the skipping variant when `mode` is set,
// with kSkipGroupTiles light tiles per wave when `grouped` is also set.
template <bool MIRROR, bool SHADOW>
void launch_sor_class(const TileView& tv, const fj_graph* g, const SorState& S, const int* prev, int* cur,
                      const SolveLayout& L, const int* mode, hipStream_t st, bool grouped = false) {
    const unsigned grid = waves_to_blocks(tv.nchunks + tv.ntiles);
    if (mode && grouped)
        hipLaunchKernelGGL((k_sor_class<MIRROR, SHADOW, true, kSkipGroupTiles>),
                           dim3(waves_to_blocks(tv.nchunks + (tv.ntiles + kSkipGroupTiles - 1) / kSkipGroupTiles)),
                           dim3(kBlock), 0, st, tv, g->prow_ptr, g->pcol, g->pw, S, prev, cur, L.bad, L.stats, mode);
    else if (mode)
        hipLaunchKernelGGL((k_sor_class<MIRROR, SHADOW, true>), dim3(grid), dim3(kBlock), 0, st, tv, g->prow_ptr,
                           g->pcol, g->pw, S, prev, cur, L.bad, L.stats, mode);
    else
        hipLaunchKernelGGL((k_sor_class<MIRROR, SHADOW, false>), dim3(grid), dim3(kBlock), 0, st, tv, g->prow_ptr,
                           g->pcol, g->pw, S, prev, cur, L.bad, L.stats, static_cast<const int*>(nullptr));
}

fj_status solve_sor(const fj_graph* g, const double* s, const fj_solve_opts* o, double epsp, double* z,
                    const SolveLayout& L, fj_solve_stats* out, hipStream_t st, int64_t cap) {
    const int64_t n = g->n;
    const int bs = 256;
    FJ_HIP(hipMemsetAsync(L.hacc, 0, sizeof(unsigned long long) * (2 * g->tiles_p.nheavy + 2), st));
    FJ_HIP(hipMemsetAsync(L.zmax_bits, 0, sizeof(unsigned long long), st));
    if (n > 0)
        hipLaunchKernelGGL(k_sor_init, dim3(std::min<unsigned>(grid1d(n, bs), 2048u)), dim3(bs), 0, st, n, g->perm, s,
                           o->z0, o->c, L.sp, L.zh, L.zq, L.bad, L.zmax_bits);
    int hbad = 0;
    unsigned long long hzmax = 0;
    FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipMemcpyAsync(&hzmax, L.zmax_bits, sizeof(hzmax), hipMemcpyDeviceToHost, st));
    FJ_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("s must be finite and >= 0, and z0 finite");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const int K = o->check_every > 0 ? o->check_every : 8;
    const int max_ref = o->max_refinements >= 0 ? o->max_refinements : 8;
    const int nc = g->num_colours;
    std::vector<TileView> views(nc);
    for (int k = 0; k < nc; ++k) views[k] = tile_view(g->tiles_p, k);
    int64_t sweeps = 0, launches = 0, mirror_sweeps = 0;
    int64_t d_blocks = 0;  // opts.measures: D's block sums from the last certificate
    int refinements = 0;
    bool converged = false, capped = false, diverged = false;
    double max_ratio = 0.0;
    std::vector<int> hf(K);
    LaunchTimer timer;
    timer.on = o->profile != 0;
    timer.st = st;
    // persistent cooperative launch when the device allows it
    int coop_grid = 0;
    if (n > 0 && o->persistent) {
        int dev = 0, coop = 0, cus = 0, occ = 0;
        FJ_HIP(hipGetDevice(&dev));
        FJ_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        FJ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        FJ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sor_persistent, kPBlock, 0));
        if (coop && cus > 0 && occ > 0) coop_grid = cus * occ;
    }
    SorArgs sa{};
    sa.tile_start = g->tiles_p.tile_start;
    sa.tile_heavy = g->tiles_p.tile_heavy;
    sa.heavy_row = g->tiles_p.heavy_row;
    sa.seg_tile = g->tiles_p.d_seg_tile;
    sa.seg_heavy = g->tiles_p.d_seg_heavy;
    sa.ncls = nc;
    sa.prow_ptr = g->prow_ptr;
    sa.pcol = g->pcol;
    sa.pw = g->pw;
    // FP64 sweeps: the margin of 1e-6 h keeps a quiet sweep certified under the
    // FP64 rounding of the standalone certificate (different summation order).
    SorState S64{L.sp, g->popd, g->pinv64, L.zh, L.zq, o->omega, 1.0 - 1e-6, epsp, L.hacc, L.zmax_bits,
                 L.zsh, L.zqsh, 0};
    S64.brow = g->directed ? g->qrow_ptr : g->prow_ptr;
    S64.bcol = g->directed ? g->qcol : g->pcol;
    S64.bw = g->directed ? g->qw : g->pw;
    // Merged tail: the trailing small classes [merge_T, nc) are swept by one
    // launch in which their rows see each other's values from before it (a
    // Jacobi step among them).  With A = (I+D) - W, the sweep is the splitting
    // A = M - N with M = (I+D)/omega - E (E: couplings to earlier rows); by the
    // Householder-John theorem it converges for symmetric positive definite A
    // when M + M^T - A = (2/omega - 1)(I+D) + W_tail is positive definite,
    // which holds when every merged row's coupling to the merged rows is below
    // (2/omega - 1) of 1 + d_i (diagonal dominance).  A 10% margin is kept.
    int merge_T = nc;
    if (!o->no_tail_merge && !g->directed && g->merge_min < nc) {
        const double lim = 0.9 * (2.0 / o->omega - 1.0);
        for (int t = g->merge_min; t < nc - 1; ++t)
            if (g->merge_coupling[t] < lim) { merge_T = t; break; }
    }
    TileView tail{};
    if (merge_T < nc) {
        const TileSet& T = g->tiles_p;
        tail = tile_view_all(T);
        tail.t0 = T.seg_tile[merge_T];
        tail.ntiles = T.seg_tile[nc] - T.seg_tile[merge_T];
        tail.c0 = T.seg_chunk[merge_T];
        tail.nchunks = T.seg_chunk[nc] - T.seg_chunk[merge_T];
        tail.h0 = T.seg_heavy[merge_T];
        tail.h1 = T.seg_heavy[nc];
        S64.sh_base = g->class_off[merge_T];
    }
    const int64_t tail_rows = merge_T < nc ? n - g->class_off[merge_T] : 0;
    // Fixed-point sweeps: light rows gather the 32-bit copy, whose error per
    // arc is <= 4.7e-10; a 5% margin on h makes it likely that the FP64
    // certificate holds when these sweeps go quiet.  FP64 sweeps follow if not.
    SorState SMIR = S64;
    SMIR.thr = 0.95;
    bool mirror = o->precision == FJ_FP32 && o->gather_bits != 64 && fix_range_ok(hzmax);
    sa.S = S64;
    sa.bad = L.bad;
    sa.stats = L.stats;
    sa.gs.counter = L.barrier;
    sa.gs.abort = L.abort;
    const int KP = std::max(K, 32);
    std::vector<int> hfp(KP);
    // Bound skipping: an update raises the bounds of the rows of A that read
    // the updated value, through the updated row's arcs in CSR(A) (symmetric
    // pattern) or in the relabelled CSR(A^T) (directed); every class must run
    // in k_sor_class (which keeps the bounds).  Considered from the second sweep of each phase (fixed-point
    // sweeps, FP64 sweeps, each refinement), once a sweep updated fewer than
    // `limit` rows.
    bool skipping = o->skip_below >= 0.0 && n > 0 && S64.brow != nullptr &&
                    (o->skip_below > 0.0 || g->nnz >= kSkipMinArcs);
    for (int k = 0; k < nc && skipping; ++k)
        if (!g->class_packed[k]) skipping = false;
    const double limit = (o->skip_below > 0.0 ? o->skip_below : kSkipBelow) * static_cast<double>(n);
    std::vector<int> hmodes(K, 0);
    // The first batch of sweeps of each phase runs the plain kernel (every row
    // updates early on); the batches after it run the skipping variant, whose
    // mode k_sweep_begin sets per sweep from the update counts.
    while (true) {
        bool quiet = false;
        bool skip_batch = false;      // this batch runs the skipping variant
        bool grouped = false;         // ... with grouped light tiles (the last sweep skipped)
        int64_t phase_start = -1;     // first sweep of this phase in per-class launches
        while (!quiet && coop_grid > 0 && !mirror) {
            if (sweeps + KP > kMaxRounds || (sweeps + KP) * (g->nnz + n) > cap) break;
            FJ_HIP(hipMemsetAsync(L.flags + sweeps, 0, sizeof(int) * KP, st));
            FJ_HIP(hipMemsetAsync(L.barrier, 0, sizeof(unsigned), st));
            FJ_HIP(hipMemsetAsync(L.abort, 0, sizeof(int), st));
            sa.max_sweeps = KP;
            sa.flags = L.flags + sweeps;
            void* args[] = {&sa};
            fj_status rc0 = timer.before();
            if (rc0) return rc0;
            FJ_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_sor_persistent), dim3(coop_grid),
                                              dim3(kPBlock), args, 0, st));
            rc0 = timer.after();
            if (rc0) return rc0;
            ++launches;
            int habort = 0;
            FJ_HIP(hipMemcpyAsync(hfp.data(), L.flags + sweeps, sizeof(int) * KP, hipMemcpyDeviceToHost, st));
            FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
            FJ_HIP(hipMemcpyAsync(&habort, L.abort, sizeof(int), hipMemcpyDeviceToHost, st));
            FJ_HIP(hipStreamSynchronize(st));
            if (hbad) { diverged = true; break; }
            int used = KP;
            for (int b = 0; b < KP; ++b)
                if (hfp[b] == 0) { used = b + 1; quiet = true; break; }
            if (habort) {  // a barrier timed out: continue with per-class launches
                coop_grid = 0;
                quiet = false;
                used = KP;
                for (int b = 0; b < KP; ++b)
                    if (hfp[b] == 0) { used = b; break; }
            }
            sweeps += used;
        }
        if (diverged) break;
        while (!quiet) {
            if (sweeps + K > kMaxRounds || (sweeps + K) * (g->nnz + n) > cap) { capped = true; break; }
            if (phase_start < 0) phase_start = sweeps;
            FJ_HIP(hipMemsetAsync(L.flags + sweeps, 0, sizeof(int) * K, st));
            for (int b = 0; b < K; ++b) {
                int* cur = L.flags + sweeps + b;
                const int* prev = b > 0 ? cur - 1 : nullptr;
                SorState SW = mirror ? SMIR : S64;
                const int* mode = nullptr;
                if (skip_batch) {
                    mode = L.modes + sweeps + b;
                    SW.ub = L.ub;
                    SW.ub_tail = L.ub_tail;
                    const int64_t tail_start = merge_T < nc ? g->class_off[merge_T] : n;
                    hipLaunchKernelGGL(k_sweep_begin,
                                       dim3(std::max<int64_t>(1, std::min<int64_t>(grid1d(n - tail_start, bs), 256))),
                                       dim3(bs), 0, st, prev, sweeps + b, L.ub, L.ub_tail, tail_start, n, L.stats,
                                       L.snaps, L.modes, sweeps + b > phase_start ? 1 : 0, limit);
                    ++launches;
                } else if (skipping) {
                    hipLaunchKernelGGL(k_sweep_snap, dim3(1), dim3(64), 0, st, prev, sweeps + b, L.stats, L.snaps,
                                       L.modes);
                    ++launches;
                }
                for (int k = 0; k < merge_T; ++k) {
                    const TileView& tv = views[k];
                    if (tv.ntiles == 0) continue;
                    fj_status rc0 = timer.before();
                    if (rc0) return rc0;
                    const SorState& S = SW;
                    if (g->class_packed[k]) {
                        if (mirror) launch_sor_class<true, false>(tv, g, S, prev, cur, L, mode, st, grouped);
                        else launch_sor_class<false, false>(tv, g, S, prev, cur, L, mode, st, grouped);
                        ++launches;
                    } else {
                        const unsigned grid = waves_to_blocks(tv.nchunks + tv.ntiles);
                        if (mirror)
                            hipLaunchKernelGGL(k_sor_tiles<true>, dim3(grid), dim3(kBlock), 0, st, tv, g->prow_ptr,
                                               g->pcol, g->pw, S, L.partial, prev, cur, L.bad, L.stats);
                        else
                            hipLaunchKernelGGL(k_sor_tiles<false>, dim3(grid), dim3(kBlock), 0, st, tv, g->prow_ptr,
                                               g->pcol, g->pw, S, L.partial, prev, cur, L.bad, L.stats);
                        ++launches;
                        if (tv.h1 > tv.h0) {
                            hipLaunchKernelGGL(k_sor_heavy, dim3(waves_to_blocks(tv.h1 - tv.h0)), dim3(kBlock), 0,
                                               st, tv, S, L.partial, prev, cur, L.bad, L.stats);
                            ++launches;
                        }
                    }
                    rc0 = timer.after();
                    if (rc0) return rc0;
                }
                if (merge_T < nc) {  // the merged tail, then its commit
                    fj_status rc0 = timer.before();
                    if (rc0) return rc0;
                    const SorState& S = SW;
                    if (mirror) launch_sor_class<true, true>(tail, g, S, prev, cur, L, mode, st, grouped);
                    else launch_sor_class<false, true>(tail, g, S, prev, cur, L, mode, st, grouped);
                    hipLaunchKernelGGL(k_sor_commit, dim3(grid1d(tail_rows, bs)), dim3(bs), 0, st,
                                       g->class_off[merge_T], n, L.zsh, L.zqsh, L.zh, L.zq, prev);
                    launches += 2;
                    rc0 = timer.after();
                    if (rc0) return rc0;
                }
            }
            FJ_HIP(hipMemcpyAsync(hf.data(), L.flags + sweeps, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            FJ_HIP(hipMemcpyAsync(&hbad, L.bad, sizeof(int), hipMemcpyDeviceToHost, st));
            if (skip_batch)
                FJ_HIP(hipMemcpyAsync(hmodes.data(), L.modes + sweeps, sizeof(int) * K, hipMemcpyDeviceToHost, st));
            FJ_HIP(hipStreamSynchronize(st));
            if (hbad) { diverged = true; break; }
            int used = K;
            for (int b = 0; b < K; ++b)
                if (hf[b] == 0) { used = b + 1; quiet = true; break; }
            sweeps += used;
            if (mirror) mirror_sweeps += used;
            if (trace_on()) {
                HostStats hs;
                fj_status rc0 = read_stats(L, st, &hs);
                if (rc0) return rc0;
                trace_batch("sor", mirror ? (skip_batch ? "fixed-point skipping" : "fixed-point")
                                          : (skip_batch ? "fp64 skipping" : "fp64"),
                            sweeps, used, hs);
            }
            // a batch whose last sweep skipped is followed by the grouped launches
            if (skipping) grouped = skip_batch && hmodes[used - 1] == 2;
            if (skipping) skip_batch = true;
            if (n == 0) quiet = true;
        }
        if (capped || diverged) break;
        // the last sweep changed nothing, so its residuals were final; confirm in the original labels
        if (n > 0) hipLaunchKernelGGL(k_sor_unshift, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, g->perm, L.zh, o->c, z, L.zh2);
        long long viol = 0;
        fj_status rc = o->measures ? certify<double, true>(g, s, o->c, o->c, epsp, L.zh2, static_cast<double*>(nullptr),
                                                           L, st, &max_ratio, &viol, &d_blocks)
                                   : certify<double>(g, s, o->c, o->c, epsp, L.zh2, static_cast<double*>(nullptr), L,
                                                     st, &max_ratio, &viol);
        if (rc) return rc;
        if (trace_on()) trace_cert("sor", sweeps, max_ratio, viol, refinements);
        if (viol == 0) { converged = true; break; }
        if (mirror) {  // finish with FP64 gathers
            mirror = false;
            continue;
        }
        if (refinements >= max_ref) break;
        ++refinements;
    }
    if (!converged) {
        if (n > 0) hipLaunchKernelGGL(k_sor_unshift, dim3(grid1d(n, bs)), dim3(bs), 0, st, n, g->perm, L.zh, o->c, z, L.zh2);
        long long viol = 0;
        fj_status rc = o->measures ? certify<double, true>(g, s, o->c, o->c, epsp, L.zh2, static_cast<double*>(nullptr),
                                                           L, st, &max_ratio, &viol, &d_blocks)
                                   : certify<double>(g, s, o->c, o->c, epsp, L.zh2, static_cast<double*>(nullptr), L,
                                                     st, &max_ratio, &viol);
        if (rc) return rc;
    }
    if (o->measures) {  // D came with the final certificate; the node passes run on z
        fj_status rc = measures_with_d(g, s, z, L.part_d, d_blocks, L.mws, st, o->measures);
        if (rc) return rc;
    }
    HostStats hs;
    fj_status rc = read_stats(L, st, &hs);
    if (rc) return rc;
    rc = timer.total_ms(&out->kernel_ms, &out->kernel_launches);
    if (rc) return rc;
    out->num_colours = nc;
    out->mirror_rounds = mirror_sweeps;
    out->merged_classes = merge_T < nc ? nc - merge_T : 0;
    out->skipped_rows = static_cast<int64_t>(hs.skipped);
    out->skipped_arcs = static_cast<int64_t>(hs.skipped_arcs_fix + hs.skipped_arcs_fp64);
    out->mirror_edge_visits = mirror_sweeps * g->nnz - static_cast<int64_t>(hs.skipped_arcs_fix);
    out->mirror_fp64_edge_visits = mirror_sweeps * g->heavy_arcs_p - static_cast<int64_t>(hs.skipped_heavy_fix);
    out->bound_adds = static_cast<int64_t>(hs.bound_adds);
    out->pushes = static_cast<int64_t>(hs.pushes);
    out->edge_visits = sweeps * g->nnz - static_cast<int64_t>(hs.skipped_arcs_fix + hs.skipped_arcs_fp64);
    out->rounds = sweeps;
    out->launches = launches;
    out->refinements = refinements;
    out->certified = converged ? 1 : 0;
    out->max_ratio = max_ratio;
    if (!converged) {
        set_error(diverged ? "over-relaxed sweeps diverged (non-finite residual)"
                           : capped ? "work cap reached before the certificate held"
                                    : "certificate failed after the refinement budget");
        return FJ_ERR_NOT_CONVERGED;
    }
    return FJ_OK;
}

struct CertLayout {
    double* partial; double* part_max; long long* part_viol; double* cert_max; long long* cert_viol;
};
CertLayout carve_cert(Carver& cv, const fj_graph* g) {
    CertLayout L{};
    int64_t nb = cert_parts(g);
    L.partial = cv.take<double>(g->tiles_a.nchunks + 1);
    L.part_max = cv.take<double>(nb);
    L.part_viol = cv.take<long long>(nb);
    L.cert_max = cv.take<double>(1);
    L.cert_viol = cv.take<long long>(1);
    return L;
}

}  // namespace

size_t certify_ws_bytes(const fj_graph* g) {
    Carver cv(nullptr);
    carve_cert(cv, g);
    return cv.bytes();
}

// tau = max_v |s_v - ((I+L) z)_v| / (s_v + c): the certificate's ratio with eps' = 1
fj_status residual_level(const fj_graph* g, const double* s, const double* z, double c, void* ws, size_t ws_bytes,
                         hipStream_t st, double* tau) {
    if (ws_bytes < certify_ws_bytes(g)) {
        set_error("residual level: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    Carver cv(ws);
    CertLayout C = carve_cert(cv, g);
    SolveLayout L{};
    L.partial = C.partial;
    L.part_max = C.part_max;
    L.part_viol = C.part_viol;
    L.cert_max = C.cert_max;
    L.cert_viol = C.cert_viol;
    long long viol = 0;
    return certify<double>(g, s, 0.0, c, 1.0, z, static_cast<double*>(nullptr), L, st, tau, &viol);
}

}  // namespace fj

using namespace fj;

extern "C" fj_status fj_certify(const fj_graph* g, const double* s, const double* z, double eps, double c,
                                double sigma, double* out_max_ratio, void* ws, size_t ws_bytes, void* stream) {
    if (!g || !out_max_ratio || !ws || ((!s || !z) && g->n > 0)) {
        set_error("fj_certify: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!(eps > 0.0 && eps < 1.0) || !(c >= 0.0) || !(sigma > 0.0)) {
        set_error("fj_certify: need eps in (0,1), c >= 0, sigma > 0");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < certify_ws_bytes(g)) {
        set_error("fj_certify: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    Carver cv(ws);
    CertLayout C = carve_cert(cv, g);
    SolveLayout L{};
    L.partial = C.partial;
    L.part_max = C.part_max;
    L.part_viol = C.part_viol;
    L.cert_max = C.cert_max;
    L.cert_viol = C.cert_viol;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // z is the unshifted estimate: the residual of the shifted system equals
    // s - (I+L) z because (I+L) 1 = 1, so c enters only through the threshold.
    const double epsp = sigma * eps / (c + sigma);
    long long viol = 0;
    return certify<double>(g, s, 0.0, c, epsp, z, static_cast<double*>(nullptr), L, st, out_max_ratio, &viol);
}

extern "C" size_t fj_solve_workspace_bytes(const fj_graph* g, const fj_solve_opts* opts) {
    if (!g || !opts) return 0;
    Carver cv(nullptr);
    carve_solve(cv, g, opts->precision, opts->push_scatter == 2);
    return cv.bytes();
}

extern "C" fj_status fj_solve(const fj_graph* g, const double* s, const fj_solve_opts* o, double* z, void* ws,
                              size_t ws_bytes, fj_solve_stats* stats, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!g || !o || !z || !ws || (!s && g->n > 0)) {
        set_error("fj_solve: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!(o->eps > 0.0 && o->eps < 1.0) || !(o->omega > 0.0 && o->omega < 2.0) || !(o->c >= 0.0) ||
        !(o->sigma > 0.0) || !std::isfinite(o->c) || !std::isfinite(o->sigma)) {
        set_error("fj_solve: need eps in (0,1), omega in (0,2), c >= 0, sigma > 0");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (o->precision != FJ_FP32 && o->precision != FJ_FP64) {
        set_error("fj_solve: precision must be FJ_FP32 or FJ_FP64");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    int sched = o->schedule;
    if (sched == FJ_SCHED_AUTO) sched = g->num_colours > 0 ? FJ_SCHED_SOR : FJ_SCHED_PUSH;
    if (sched == FJ_SCHED_SOR && g->num_colours == 0) {
        set_error("fj_solve: FJ_SCHED_SOR needs a graph created with FJ_GRAPH_COLOUR");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (sched == FJ_SCHED_PUSH && o->omega > 1.0) {
        set_error("fj_solve: concurrent push rounds need omega <= 1 (over-relaxation needs FJ_SCHED_SOR)");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (sched != FJ_SCHED_PUSH && sched != FJ_SCHED_SOR) {
        set_error("fj_solve: unknown schedule");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (o->push_scatter < 0 || o->push_scatter > 2) {
        set_error("fj_solve: push_scatter must be 0, 1 or 2");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    Carver cv(ws);
    SolveLayout L = carve_solve(cv, g, o->precision, o->push_scatter == 2);
    if (cv.bytes() > ws_bytes) {
        set_error("fj_solve: workspace too small: need " + std::to_string(cv.bytes()) + " bytes");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    FJ_HIP(hipMemsetAsync(L.stats, 0, sizeof(unsigned long long) * kStripes * kStripeStride, st));
    FJ_HIP(hipMemsetAsync(L.bad, 0, sizeof(int), st));
    const int one = 1;
    FJ_HIP(hipMemcpyAsync(L.one, &one, sizeof(int), hipMemcpyHostToDevice, st));
    const double epsp = o->sigma * o->eps / (o->c + o->sigma);
    const int64_t cap = o->max_edge_visits > 0 ? o->max_edge_visits : 4096 * (g->nnz + g->n);
    fj_solve_stats local{};
    fj_status rc;
    if (sched == FJ_SCHED_SOR)
        rc = solve_sor(g, s, o, epsp, z, L, &local, st, cap);
    else if (o->push_scatter == 2)
        rc = o->precision == FJ_FP64 ? solve_push_frontier<double>(g, s, o, epsp, z, L, &local, st, cap)
                                     : solve_push_frontier<float>(g, s, o, epsp, z, L, &local, st, cap);
    else if (!o->push_scatter && g->a_packed)
        rc = solve_rounds_gather(g, s, o, epsp, z, L, &local, st, cap);
    else if (o->precision == FJ_FP64)
        rc = solve_push<double>(g, s, o, epsp, z, L, &local, st, cap);
    else
        rc = solve_push<float>(g, s, o, epsp, z, L, &local, st, cap);
    if (o->measures && sched != FJ_SCHED_SOR && (rc == FJ_OK || rc == FJ_ERR_NOT_CONVERGED)) {
        const fj_status mrc = measures_full(g, s, z, L.mws, st, o->measures);
        if (mrc != FJ_OK) rc = mrc;
    }
    local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = local;
    return rc;
}

extern "C" fj_status fj_tune_omega(const fj_graph* g, const double* s, const fj_solve_opts* opts,
                                   const double* omegas, int32_t n_omegas, int64_t* updates, double* seconds,
                                   double* best_omega, double* z, void* ws, size_t ws_bytes, void* stream) {
    if (!g || !opts || !omegas || n_omegas < 1 || !best_omega) {
        set_error("fj_tune_omega: null argument or no candidates");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    int64_t best_updates = -1;
    double best = 1.0;
    for (int32_t k = 0; k < n_omegas; ++k) {
        fj_solve_opts o = *opts;
        o.omega = omegas[k];
        o.profile = 0;
        o.measures = nullptr;  // the candidates' measures are not wanted
        fj_solve_stats st{};
        fj_status rc = fj_solve(g, s, &o, z, ws, ws_bytes, &st, stream);
        if (rc != FJ_OK && rc != FJ_ERR_NOT_CONVERGED) return rc;
        const int64_t u = rc == FJ_OK ? st.pushes : -1;
        if (updates) updates[k] = u;
        if (seconds) seconds[k] = st.seconds;
        if (u >= 0 && (best_updates < 0 || u < best_updates || (u == best_updates && omegas[k] < best))) {
            best_updates = u;
            best = omegas[k];
        }
    }
    if (best_updates < 0) {
        set_error("fj_tune_omega: no candidate reached the certificate");
        return FJ_ERR_NOT_CONVERGED;
    }
    *best_omega = best;
    return FJ_OK;
}
