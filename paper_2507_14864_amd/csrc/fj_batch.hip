// Batched solve: many graphs and many opinion vectors per graph in one
// enqueued sequence with device-side convergence, recordable as a hipGraph.
//
// Every vector is solved by the same colour-ordered ImprovedBLISOR sweeps as
// fj_solve (Alg. 2 around Alg. 3, Eqs. (sor1)-(sor3), Thm. 8), in FP64, and
// judged by the same certificate (Lemma 7 with Alg. 2's shift).
//  - Items with k = 1 are joined into one block-diagonal graph.  Its colour
//    classes are the union of the components' classes, so one launch per
//    class serves every component; a component whose last sweep updated
//    nothing has final residuals (components do not interact) and is skipped.
//  - Items with k > 1 keep their vectors node-major ([n][k]); a wave owns a
//    row and lane l owns vector l, so every arc reads k estimates with one
//    coalesced access.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fj_device.h"
#include "fj_internal.h"
#include "fj_sor.h"
#include "fj_tile.h"

// one row of the caller-bound copy tables
struct fj_batch_copy {
    const double* src;
    double* dst;
    int64_t count;
};

namespace fj {
namespace {

inline unsigned g1d(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

// ------------------------------------------------------------ union build
__global__ void k_item_rowptr_check(int64_t n, int64_t nnz, const int32_t* __restrict__ rp, int* err) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > n) return;
    int32_t v = rp[i];
    bool bad = v < 0 || v > nnz || (i == 0 && v != 0) || (i == n && v != nnz) || (i < n && rp[i + 1] < v);
    if (bad) atomicOr(err, 1);
}

__global__ void k_union_copy(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const float* __restrict__ w, int64_t noff, int64_t aoff, int comp, int32_t* urp,
                             int32_t* ucol, float* uw, int32_t* comp_of, int* err) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    urp[noff + i] = static_cast<int32_t>(aoff + rp[i]);
    comp_of[noff + i] = comp;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        int32_t j = col[e];
        if (j < 0 || j >= n) atomicOr(err, 2);  // must stay inside its own component
        ucol[aoff + e] = static_cast<int32_t>(noff + j);
        if (uw) uw[aoff + e] = w ? w[e] : 1.0f;
    }
}

// symmetry of the undirected components (the union itself is declared directed)
__global__ void k_union_symmetry(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const float* __restrict__ w, const int32_t* __restrict__ comp_of,
                                 const int32_t* __restrict__ comp_dir, int* err) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n || comp_dir[comp_of[i]]) return;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        int j = col[k];
        int64_t lo = rp[j], hi = rp[j + 1] - 1, found = -1;
        while (lo <= hi) {
            int64_t mid = (lo + hi) >> 1;
            int cc = col[mid];
            if (cc == i) { found = mid; break; }
            if (cc < i) lo = mid + 1; else hi = mid - 1;
        }
        if (found < 0 || (w && w[found] != w[k])) {
            atomicOr(err, 4);
            return;
        }
    }
}

__global__ void k_gather_i32(int64_t n, const int32_t* __restrict__ idx, const int32_t* __restrict__ src,
                             int32_t* dst) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// --------------------------------------------------------- flags per slot
// slot = one component of the union or one multi-vector item
__global__ void k_flags_reset(int nslots, int* upd, int* done, int* sweeps_done, int* all_done, int* bad,
                              unsigned long long* vupd, unsigned long long* vdone, int* vsw) {
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        upd[s] = 0;
        done[s] = 0;
        sweeps_done[s] = 0;
        vupd[s] = 0ull;
        vdone[s] = 0ull;
    }
    for (int q = threadIdx.x; q < 64 * nslots; q += blockDim.x) vsw[q] = 0;
    if (threadIdx.x == 0) {
        all_done[0] = all_done[1] = 0;
        *bad = 0;
    }
}

// vupd/vdone (multi-vector items): bit l set when vector l updated in this
// sweep / had a sweep without an update.  The vectors of an item are
// independent systems on one graph, so a vector whose sweep changed nothing
// is converged: its lane stops gathering (bit for bit the same result).
// Slots [s0, s1) are one branch (the union's components, or the multi-vector
// items), whose launches all test that branch's all_done flag.
__global__ __launch_bounds__(256) void k_sweep_end(int s0, int s1, int sweep, int* upd, int* done, int* sweeps_done,
                                                   int* all_done, unsigned long long* vupd, unsigned long long* vdone,
                                                   int* vsw) {
    __shared__ int s_open;
    if (threadIdx.x == 0) s_open = 0;
    __syncthreads();
    if (*all_done) return;
    int open = 0;
    for (int s = s0 + static_cast<int>(threadIdx.x); s < s1; s += blockDim.x) {
        if (!done[s]) {
            if (!upd[s]) {
                done[s] = 1;
                sweeps_done[s] = sweep + 1;
            } else {
                open = 1;
            }
        }
        upd[s] = 0;
        for (unsigned long long fresh = ~vupd[s] & ~vdone[s]; fresh; fresh &= fresh - 1)
            vsw[64 * s + __builtin_ctzll(fresh)] = sweep + 1;
        vdone[s] |= ~vupd[s];
        vupd[s] = 0ull;
    }
    if (open) s_open = 1;
    __syncthreads();
    if (threadIdx.x == 0 && !s_open) *all_done = 1;
}

// ------------------------------------------------- union sweep (k = 1)
// Heavy rows finish in the launch that sums their chunks.  A chunk wave
// publishes its partial with returning atomic exchanges, which are performed
// where every CU sees them (the chunk waves of one row run on any XCD, and
// plain stores would stay in this XCD's L2), then counts its arrival on the
// row's counter once every lane's exchange has returned: the counter's
// address depends on the returned values.  The wave whose arrival completes
// a multiple of the row's chunk count reads the partials back the same way
// and adds them in chunk order, as a separate finishing launch would.  The
// counters are cleared when a solve starts.
__device__ __forceinline__ int after_all_lanes(unsigned long long v) {
    const unsigned long long m = __ballot(v == 0x7ff4dead0badf00dull);  // every lane's v
    int dep;
    __asm__ volatile("v_mov_b32 %0, 0 ; after %1" : "=v"(dep) : "v"(static_cast<unsigned>(m)));
    return dep;
}
__device__ __forceinline__ unsigned long long publish_ret(double* p, double v) {
    return atomicExch(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(__double_as_longlong(v)));
}
__device__ __forceinline__ double read_published(double* p) {
    return __longlong_as_double(static_cast<long long>(atomicOr(reinterpret_cast<unsigned long long*>(p), 0ull)));
}

__global__ void k_fill_i32(int64_t count, int32_t* p, int32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// NCH: 64-arc chunks of a light tile in flight per step (a tuned launch
// parameter; the sums are added in arc order whatever its value)
template <int NCH>
__global__ __launch_bounds__(kBlock) void k_usor_tiles(TileView tv, const int32_t* __restrict__ prow_ptr,
                                                       const int32_t* __restrict__ pcol, const float* __restrict__ pw,
                                                       SorState S, double* partial, int32_t* hcnt,
                                                       const int32_t* __restrict__ pcomp,
                                                       const double* __restrict__ comp_omega, int* upd,
                                                       const int* __restrict__ done,
                                                       const int* __restrict__ all_done, int* bad) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    if (*all_done) return;
    const int wid = wave_id(), lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    const double* __restrict__ zh = S.zh;
    auto arc = [&](int k) {
        double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
        return a * zh[__builtin_nontemporal_load(&pcol[k])];
    };
    if (wv < tv.nchunks) {  // a chunk of a heavy row; the last one finishes the row
        const int64_t cidx = tv.c0 + wv;
        const int32_t h = tv.chunk_heavy[cidx];
        const int32_t row = tv.heavy_row[h];
        const int c = pcomp[row];
        if (done[c]) return;
        const int beg = tv.chunk_beg[cidx];
        const int end = min(beg + kArcBudget, prow_ptr[row + 1]);
        const double part = chunk_sum(beg, end, arc);
        unsigned long long ret = 0;
        if (lane == 0) ret = publish_ret(partial + cidx, part);
        const int dep = after_all_lanes(ret);
        int old = 0;
        if (lane == 0) old = atomicAdd(hcnt + h + dep, 1);
        old = __shfl(old, 0, 64);
        const int32_t q0 = tv.heavy_chunk0[h], q1 = tv.heavy_chunk0[h + 1];
        if ((old + 1) % (q1 - q0) != 0) return;
        double sum = 0.0;
        for (int32_t q = q0 + lane; q < q1; q += 64) sum += read_published(partial + q);
        sum = wave_sum(sum);
        if (lane == 0) {
            bool nf = false;
            SorState Sc = S;
            Sc.omega = comp_omega[c];
            if (sor_row(row, sum, Sc, &nf)) flag_set(&upd[c]);
            if (nf) flag_set(bad);
        }
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    const int c0 = pcomp[r0], c1 = pcomp[r0 + nrows - 1];
    if (c1 - c0 <= 1 && done[c0] && done[c1]) return;
    double sum = tile_row_sums<NCH>(prow_ptr, r0, nrows, s_pre[wid], s_acc[wid], arc);
    if (lane < nrows) {
        const int c = pcomp[r0 + lane];
        if (!done[c]) {
            bool nf = false;
            SorState Sc = S;
            Sc.omega = comp_omega[c];
            if (sor_row(r0 + lane, sum, Sc, &nf)) flag_set(&upd[c]);
            if (nf) flag_set(bad);
        }
    }
}

// ------------------------------------------- multi-vector sweep (k > 1)
struct MState {
    const double* sp;    // [n][k] s' = s + c, relabelled rows
    const double* popd;  // [n] 1 + d
    const double* pinv;  // [n] 1 / (1 + d)
    double* zh;          // [n][k]
    double omega, thr, epsp;
    int k;
    const unsigned long long* vdone;  // the item's converged vectors (bit per lane)
    unsigned long long* vupd;         // the item's vectors updated in this sweep
};
// set the bits of m in *mask; the read first keeps the waves of a sweep from
// all contending for the one word once its bits are set
__device__ __forceinline__ void vmask_or(unsigned long long* mask, unsigned long long m) {
    if (m & ~__atomic_load_n(mask, __ATOMIC_RELAXED)) atomicOr(mask, m);
}
// lane l sweeps vector l while it is not converged
__device__ __forceinline__ bool mrhs_active(const MState& S, int l) {
    return l < S.k && !((*S.vdone >> l) & 1ull);
}

// active lane l: sum over arcs [beg, end) of a_e * zh[col_e][l], U arcs in
// flight (a tuned launch parameter); added in arc order whatever U is.  The
// arc range is the same in every lane: taken into scalar registers, the
// column indices (and weights) arrive by scalar loads, the next U while the
// current U gathers are in flight, and each gather is one coalesced row of k
// values.  The last fewer than U arcs go in one step of B arcs (B the
// smallest power of two >= their count), the indices past the end clamped to
// the last arc and left out of the sum.
template <int B, bool W>
__device__ __forceinline__ double mrhs_arc_tail(double acc, int e, int end, const int32_t* __restrict__ pcol,
                                                const float* __restrict__ pw, const double* __restrict__ zl, int k) {
    int j[B];
    float a[B];
    double v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
        const int q = min(e + u, end - 1);
        j[u] = pcol[q];
        a[u] = W ? pw[q] : 1.0f;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = zl[static_cast<int64_t>(j[u]) * k];
#pragma unroll
    for (int u = 0; u < B; ++u)
        if (e + u < end) acc += static_cast<double>(a[u]) * v[u];
    return acc;
}
template <int U, bool W>
__device__ __forceinline__ double mrhs_arc_sum_w(int beg, int end, const int32_t* __restrict__ pcol,
                                                 const float* __restrict__ pw, const double* __restrict__ zl, int k) {
    double acc = 0.0;
    int e = beg;
    if (e + U <= end) {
        int jn[U];
        float an[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            jn[u] = pcol[e + u];
            an[u] = W ? pw[e + u] : 1.0f;
        }
        while (true) {
            double v[U];
            float a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                v[u] = zl[static_cast<int64_t>(jn[u]) * k];
                a[u] = an[u];
            }
            e += U;
            const bool more = e + U <= end;
            if (more) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    jn[u] = pcol[e + u];
                    an[u] = W ? pw[e + u] : 1.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += static_cast<double>(a[u]) * v[u];
            if (!more) break;
        }
    }
    const int rem = end - e;  // 0 <= rem < U
    if (rem <= 0) return acc;
    if (U > 8 && rem > 8) return mrhs_arc_tail<(U > 8 ? 16 : 1), W>(acc, e, end, pcol, pw, zl, k);
    if (U > 4 && rem > 4) return mrhs_arc_tail<(U > 4 ? 8 : 1), W>(acc, e, end, pcol, pw, zl, k);
    if (rem > 2) return mrhs_arc_tail<4, W>(acc, e, end, pcol, pw, zl, k);
    if (rem > 1) return mrhs_arc_tail<2, W>(acc, e, end, pcol, pw, zl, k);
    return mrhs_arc_tail<1, W>(acc, e, end, pcol, pw, zl, k);
}
template <int U>
__device__ __forceinline__ double mrhs_arc_sum(int beg, int end, const int32_t* __restrict__ pcol,
                                               const float* __restrict__ pw, const double* __restrict__ zh, int k,
                                               int l, bool act) {
    beg = __builtin_amdgcn_readfirstlane(beg);
    end = __builtin_amdgcn_readfirstlane(end);
    if (!act) return 0.0;
    return pw ? mrhs_arc_sum_w<U, true>(beg, end, pcol, pw, zh + l, k)
              : mrhs_arc_sum_w<U, false>(beg, end, pcol, pw, zh + l, k);
}

// the update of row i, vector l, with zhat'[i][l] and s'[i][l] already loaded
__device__ __forceinline__ bool mrhs_row_with(int64_t i, int l, double sum, const MState& S, double z, double sp,
                                              bool* nf, bool act) {
    if (!act) return false;
    const int64_t q = i * S.k + l;
    double r = sp - S.popd[i] * z + sum;
    *nf = !isfinite(r);
    if (fabs(r) > S.thr * S.epsp * sp) {
        S.zh[q] = z + S.omega * r * S.pinv[i];
        return true;
    }
    return false;
}
__device__ __forceinline__ bool mrhs_row(int64_t i, int l, double sum, const MState& S, bool* nf, bool act) {
    if (!act) return false;
    const int64_t q = i * S.k + l;
    double z = S.zh[q], sp = S.sp[q];
    double r = sp - S.popd[i] * z + sum;
    *nf = !isfinite(r);
    if (fabs(r) > S.thr * S.epsp * sp) {
        S.zh[q] = z + S.omega * r * S.pinv[i];
        return true;
    }
    return false;
}

template <int U>
__global__ __launch_bounds__(kBlock) void k_msor_class(TileView tv, int64_t rb, int64_t re,
                                                       const int32_t* __restrict__ prow_ptr,
                                                       const int32_t* __restrict__ pcol, const float* __restrict__ pw,
                                                       MState S, double* partial, int32_t* hcnt, int* upd,
                                                       const int* __restrict__ done, const int* __restrict__ all_done,
                                                       int* bad) {
    if (*all_done || *done) return;
    const int wid = wave_id(), lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (wv < tv.nchunks) {  // a chunk of a heavy row; the last one finishes the row
        const int64_t cidx = tv.c0 + wv;
        const int32_t h = tv.chunk_heavy[cidx];
        const int32_t row = tv.heavy_row[h];
        const int beg = tv.chunk_beg[cidx];
        const int end = min(beg + kArcBudget, prow_ptr[row + 1]);
        const bool act = mrhs_active(S, lane);
        const double acc = mrhs_arc_sum<U>(beg, end, pcol, pw, S.zh, S.k, lane, act);
        unsigned long long ret = 0;
        if (lane < S.k) ret = publish_ret(partial + cidx * S.k + lane, acc);
        const int dep = after_all_lanes(ret);
        int old = 0;
        if (lane == 0) old = atomicAdd(hcnt + h + dep, 1);
        old = __shfl(old, 0, 64);
        const int32_t c0 = tv.heavy_chunk0[h], c1 = tv.heavy_chunk0[h + 1];
        if ((old + 1) % (c1 - c0) != 0) return;
        double sum = 0.0;
        if (act)
            for (int32_t q = c0; q < c1; ++q) sum += read_published(partial + static_cast<int64_t>(q) * S.k + lane);
        bool nf = false;
        const bool u = mrhs_row(row, lane, sum, S, &nf, act);
        const unsigned long long um = __ballot(u);
        if (um && lane == 0) {
            flag_set(upd);
            vmask_or(S.vupd, um);
        }
        if (__ballot(nf) && lane == 0) flag_set(bad);
        return;
    }
    const int64_t i = rb + (wv - tv.nchunks);
    if (i >= re) return;
    const int b = prow_ptr[i], e = prow_ptr[i + 1];
    if (e - b > kArcBudget) return;  // heavy: its chunk waves
    const bool act = mrhs_active(S, lane);
    // the row's own values load before the gathers (no row of the class
    // reads another, so nothing writes them meanwhile)
    double z = 0.0, sp = 0.0;
    if (act) {
        z = S.zh[i * S.k + lane];
        sp = S.sp[i * S.k + lane];
    }
    double acc = mrhs_arc_sum<U>(b, e, pcol, pw, S.zh, S.k, lane, act);
    bool nf = false;
    bool u = mrhs_row_with(i, lane, acc, S, z, sp, &nf, act);
    const unsigned long long um = __ballot(u);
    if (um && lane == 0) {
        flag_set(upd);
        vmask_or(S.vupd, um);
    }
    if (__ballot(nf) && lane == 0) flag_set(bad);
}

__global__ void k_minit(int64_t n, int k, const int32_t* __restrict__ perm, const double* __restrict__ s, double c,
                        double* sp, double* zh, int* bad) {
    int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= n * k) return;
    int64_t i = q / k;
    int l = static_cast<int>(q - i * k);
    double si = s[static_cast<int64_t>(perm[i]) * k + l];
    if (!(si >= 0.0) || !isfinite(si)) flag_set(bad);
    sp[q] = si + c;
    zh[q] = 0.0;
}

__global__ void k_munshift(int64_t n, int k, const int32_t* __restrict__ perm, const double* __restrict__ zh,
                           double c, double* z) {
    int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= n * k) return;
    int64_t i = q / k;
    int l = static_cast<int>(q - i * k);
    z[static_cast<int64_t>(perm[i]) * k + l] = zh[q] - c;
}

// --------------------------------------------- results: union (per row)
// Per-row FP64 quantities over the union's CSR(A) in original labels, then
// fixed-order reductions per component (one block each).
//   mode 0: ratio_i = |s_i - ((I+L) z)_i| / (eps' (s_i + c))   (certificate)
//   mode 1: d_i = sum_j a_ij (z_i - z_j)^2                      (disagreement)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_urows_tiles(TileView tv, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col, const float* __restrict__ w,
                                                        const double* __restrict__ s, const double* __restrict__ z,
                                                        const double* __restrict__ opd, double c, double epsp,
                                                        double* partial, double* out) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    const int wid = wave_id(), lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (wv < tv.nchunks) {
        const int64_t cidx = tv.c0 + wv;
        const int32_t row = tv.heavy_row[tv.chunk_heavy[cidx]];
        const double zi = z[row];
        const int beg = tv.chunk_beg[cidx];
        const int end = min(beg + kArcBudget, row_ptr[row + 1]);
        double sum = chunk_sum(beg, end, [&](int k) {
            double a = w ? static_cast<double>(w[k]) : 1.0;
            if constexpr (MODE == 0) return a * z[col[k]];
            double d = zi - z[col[k]];
            return a * d * d;
        });
        if (lane == 0) partial[cidx] = sum;
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    __shared__ double s_z[kWavesPerBlock][64];
    if (lane < nrows) s_z[wid][lane] = z[r0 + lane];
    wave_sync_lds();
    const int* pre = s_pre[wid];
    double sum = tile_row_sums(row_ptr, r0, nrows, s_pre[wid], s_acc[wid], [&](int k) {
        double a = w ? static_cast<double>(w[k]) : 1.0;
        if constexpr (MODE == 0) return a * z[col[k]];
        // row of arc k inside the tile
        int slot = tile_find(pre, nrows, k - row_ptr[r0]);
        double d = s_z[wid][slot] - z[col[k]];
        return a * d * d;
    });
    if (lane < nrows) {
        const int64_t i = r0 + lane;
        if constexpr (MODE == 0) {
            double r = s[i] - opd[i] * z[i] + sum;
            out[i] = fabs(r) / (epsp * (s[i] + c));
        } else {
            out[i] = sum;
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_urows_heavy(TileView tv, const double* __restrict__ s,
                                                        const double* __restrict__ z, const double* __restrict__ opd,
                                                        double c, double epsp, const double* __restrict__ partial,
                                                        double* out) {
    const int wid = wave_id(), lane = lane_id();
    const int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (hh >= tv.h1) return;
    const int32_t c0 = tv.heavy_chunk0[hh], c1 = tv.heavy_chunk0[hh + 1];
    double sum = 0.0;
    for (int32_t q = c0 + lane; q < c1; q += 64) sum += partial[q];
    sum = wave_sum(sum);
    if (lane == 0) {
        const int64_t i = tv.heavy_row[hh];
        if constexpr (MODE == 0) {
            double r = s[i] - opd[i] * z[i] + sum;
            out[i] = fabs(r) / (epsp * (s[i] + c));
        } else {
            out[i] = sum;
        }
    }
}

// one block per component: [0] sum z, [1] sum z^2, [2] sum (z-s)^2, [3] sum d_i,
// [4] max ratio; second pass [5] sum (z - mean)^2
__global__ __launch_bounds__(256) void k_useg(const int64_t* __restrict__ node_off, const double* __restrict__ s,
                                              const double* __restrict__ z, const double* __restrict__ drow,
                                              const double* __restrict__ ratio, double* out, int pass) {
    __shared__ double lds[4];
    const int cidx = blockIdx.x;
    const int64_t b = node_off[cidx], e = node_off[cidx + 1];
    if (pass == 0) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, mx = 0;
        for (int64_t i = b + threadIdx.x; i < e; i += 256) {
            double zi = z[i], d = zi - s[i];
            a0 += zi;
            a1 += zi * zi;
            a2 += d * d;
            a3 += drow[i];
            double r = ratio[i];
            mx = fmax(mx, isfinite(r) ? r : INFINITY);
        }
        a0 = block_sum<256>(a0, lds);
        a1 = block_sum<256>(a1, lds);
        a2 = block_sum<256>(a2, lds);
        a3 = block_sum<256>(a3, lds);
        mx = wave_max(mx);
        __shared__ double smx[4];
        if (lane_id() == 0) smx[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = fmax(fmax(smx[0], smx[1]), fmax(smx[2], smx[3]));
            out[8 * cidx + 0] = a0;
            out[8 * cidx + 1] = a1;
            out[8 * cidx + 2] = a2;
            out[8 * cidx + 3] = a3;
            out[8 * cidx + 4] = m;
        }
    } else {
        const double mean = (e > b) ? out[8 * cidx + 0] / static_cast<double>(e - b) : 0.0;
        double a = 0;
        for (int64_t i = b + threadIdx.x; i < e; i += 256) {
            double d = z[i] - mean;
            a += d * d;
        }
        a = block_sum<256>(a, lds);
        if (threadIdx.x == 0) out[8 * cidx + 5] = a;
    }
}

// write per-item stats and measures of the union components
__global__ void k_ufinish(int ncomp, const int32_t* __restrict__ comp_item, const int32_t* __restrict__ comp_dir,
                          const int64_t* __restrict__ node_off, const int32_t* __restrict__ row_ptr,
                          const int64_t* __restrict__ metric_slot,
                          const double* __restrict__ seg, const int* __restrict__ sweeps_done, int slot0,
                          int budget, fj_solve_stats* stats, fj_metrics_out* mets) {
    int cidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= ncomp) return;
    const int it = comp_item[cidx];
    const double* o = seg + 8 * cidx;
    const int64_t n = node_off[cidx + 1] - node_off[cidx];
    fj_solve_stats st{};
    int sw = sweeps_done[slot0 + cidx];
    st.rounds = sw ? sw : budget;
    st.edge_visits = st.rounds * static_cast<int64_t>(row_ptr[node_off[cidx + 1]] - row_ptr[node_off[cidx]]);
    st.max_ratio = o[4];
    st.certified = (o[4] <= 1.0) ? 1 : 0;
    stats[it] = st;
    fj_metrics_out m;
    m.P = o[5];
    m.D = comp_dir[cidx] ? o[3] : 0.5 * o[3];
    m.I = o[2];
    m.C = o[1];
    m.mean = n ? o[0] / static_cast<double>(n) : 0.0;
    mets[metric_slot[it]] = m;
}

// -------------------------------------------- results: multi-vector item
// wave per row (grid-stride), lane l = vector l; per-block partials per lane:
// pass 0: [0] sum z, [1] sum z^2, [2] sum (z-s)^2, [3] sum_i sum_j a_ij (z_i-z_j)^2, [4] max ratio
// pass 1: [5] sum (z - mean)^2
constexpr int kMBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_mresults(int64_t n, int k, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, const float* __restrict__ w,
                                                     const double* __restrict__ opd, const double* __restrict__ s,
                                                     const double* __restrict__ z, double c, double epsp,
                                                     const double* __restrict__ means, double* part, int pass) {
    __shared__ double lds[kWavesPerBlock][64][6];
    const int wid = wave_id(), lane = lane_id();
    const int64_t W = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    double a[6] = {0, 0, 0, 0, 0, 0};
    const double mean = (pass == 1 && lane < k) ? means[lane] : 0.0;
    // the row is wave-uniform: its arc range and column indices come by
    // scalar loads, kU value rows in flight per step, added in arc order
    constexpr int kU = 8;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid; i < n; i += W) {
        if (lane >= k) continue;
        const double zi = z[i * k + lane];
        if (pass == 1) {
            double d = zi - mean;
            a[5] += d * d;
            continue;
        }
        const double si = s[i * k + lane];
        double sz = 0.0, sd = 0.0;
        const int end = __builtin_amdgcn_readfirstlane(row_ptr[i + 1]);
        for (int e = __builtin_amdgcn_readfirstlane(row_ptr[i]); e < end; e += kU) {
            int j[kU];
            double aw[kU], zj[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int q = min(e + u, end - 1);  // past the end: clamped, left out
                j[u] = col[q];
                aw[u] = w ? static_cast<double>(w[q]) : 1.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) zj[u] = z[static_cast<int64_t>(j[u]) * k + lane];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (e + u < end) {
                    sz += aw[u] * zj[u];
                    sd += aw[u] * (zi - zj[u]) * (zi - zj[u]);
                }
        }
        const double r = si - opd[i] * zi + sz;
        double ratio = fabs(r) / (epsp * (si + c));
        if (!isfinite(ratio)) ratio = INFINITY;
        a[0] += zi;
        a[1] += zi * zi;
        a[2] += (zi - si) * (zi - si);
        a[3] += sd;
        a[4] = fmax(a[4], ratio);
    }
    for (int q = 0; q < 6; ++q) lds[wid][lane][q] = a[q];
    __syncthreads();
    if (threadIdx.x < 64) {
        double t[6] = {0, 0, 0, 0, 0, 0};
        for (int v = 0; v < kWavesPerBlock; ++v) {
            for (int q = 0; q < 6; ++q) {
                if (q == 4) t[q] = fmax(t[q], lds[v][threadIdx.x][q]);
                else t[q] += lds[v][threadIdx.x][q];
            }
        }
        for (int q = 0; q < 6; ++q) part[(static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x) * 6 + q] = t[q];
    }
}

// one thread per vector: fixed-order reduce of the block partials
__global__ void k_mreduce(int k, int nb, const double* __restrict__ part, double* tot, double* means, int64_t n,
                          int pass) {
    const int l = threadIdx.x;
    if (l >= k) return;
    double t[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 6; ++q) {
            double v = part[(static_cast<int64_t>(b) * 64 + l) * 6 + q];
            if (q == 4) t[q] = fmax(t[q], v); else t[q] += v;
        }
    if (pass == 0) {
        for (int q = 0; q < 5; ++q) tot[8 * l + q] = t[q];
        means[l] = n ? t[0] / static_cast<double>(n) : 0.0;
    } else {
        tot[8 * l + 5] = t[5];
    }
}

__global__ void k_mfinish(int k, int item, int directed, int64_t n, int64_t nnz, int64_t mslot,
                          const double* __restrict__ tot, const int* __restrict__ sweeps_done,
                          const int* __restrict__ vsw, int slot, int budget, fj_solve_stats* stats,
                          fj_metrics_out* mets) {
    const int l = threadIdx.x;
    if (l >= k) return;
    const double* o = tot + 8 * l;
    fj_metrics_out m;
    m.P = o[5];
    m.D = directed ? o[3] : 0.5 * o[3];
    m.I = o[2];
    m.C = o[1];
    m.mean = n ? o[0] / static_cast<double>(n) : 0.0;
    mets[mslot + l] = m;
    if (l == 0) {
        double mx = 0.0;
        for (int q = 0; q < k; ++q) mx = fmax(mx, tot[8 * q + 4]);
        fj_solve_stats st{};
        int sw = sweeps_done[slot];
        st.rounds = sw ? sw : budget;
        // arcs gathered: each vector's row values over the sweeps until it went quiet
        int64_t vs = 0;
        for (int q = 0; q < k; ++q) vs += vsw[64 * slot + q] ? vsw[64 * slot + q] : st.rounds;
        st.edge_visits = vs * nnz;
        st.max_ratio = mx;
        st.certified = mx <= 1.0 ? 1 : 0;
        stats[item] = st;
    }
}

// Caller-bound inputs and outputs: row q of the table copies count doubles
// from src to dst (blockIdx.y = item).
__global__ void k_batch_copy(const fj_batch_copy* __restrict__ tab) {
    const fj_batch_copy e = tab[blockIdx.y];
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < e.count;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x)
        e.dst[q] = e.src[q];
}

// reopen the listed slots for more sweeps (their vectors too); both branch
// flags reopen (a branch with no open slot closes again at its next sweep end)
__global__ void k_reopen(int count, const int* __restrict__ slots, int* done, int* sweeps_done, int* all_done,
                         unsigned long long* vdone) {
    for (int q = threadIdx.x; q < count; q += blockDim.x) {
        const int sl = slots[q];
        done[sl] = 0;
        sweeps_done[sl] = 0;
        vdone[sl] = 0ull;
    }
    if (threadIdx.x == 0) all_done[0] = all_done[1] = 0;
}

}  // namespace
}  // namespace fj

using namespace fj;

// ---------------------------------------------------------------- host side
struct UnionGroup {
    int ncomp = 0;
    int64_t n = 0, nnz = 0;
    bool weighted = false;
    std::vector<int32_t> comp_item;
    std::vector<int64_t> node_off, arc_off;
    int32_t* row_ptr = nullptr; int32_t* col = nullptr; float* w = nullptr;
    int64_t* d_node_off = nullptr;
    int32_t* d_comp_item = nullptr; int32_t* comp_dir = nullptr; int32_t* comp_of = nullptr; int32_t* pcomp = nullptr;
    fj_graph g;
    void* gws = nullptr; size_t gws_bytes = 0;
    double* s_in = nullptr; double* z_out = nullptr;
    double* sp = nullptr; double* zh = nullptr; int32_t* zq = nullptr; double* partial = nullptr;
    int32_t* hcnt = nullptr; int64_t hcnt_len = 0;  // heavy-row arrival counters
    double* ratio = nullptr; double* drow = nullptr; double* seg = nullptr;
};

struct MrhsGroup {
    int item = 0, k = 0;
    fj_graph_desc desc{};
    fj_graph g;
    void* gws = nullptr; size_t gws_bytes = 0;
    double* s_in = nullptr; double* z_out = nullptr;
    double* sp = nullptr; double* zh = nullptr; double* partial = nullptr;
    int32_t* hcnt = nullptr; int64_t hcnt_len = 0;  // heavy-row arrival counters
    double* part = nullptr; double* tot = nullptr; double* means = nullptr;
};

struct fj_batch {
    int num_items = 0;
    std::vector<int> ks;
    std::vector<int64_t> ns;
    std::vector<int> item_group;  // -1 union, else index into M
    double eps = 0, omega = 1, c = 0, sigma = 1, epsp = 0;
    int budget = 256;
    bool concurrent = true;  // recorded graph: union and multi-vector branches concurrent
    bool has_union = false;
    UnionGroup U;
    std::vector<MrhsGroup> M;
    int nslots = 0;
    std::vector<double> slot_omega;   // relaxation factor per slot (union component or multi-vector item)
    double* d_slot_omega = nullptr;
    int* upd = nullptr; int* done = nullptr; int* sweeps_done = nullptr; int* bad = nullptr;
    int* all_done = nullptr;  // [2]: every slot of the union branch / of the multi-vector branch done
    int* vsw = nullptr;  // [nslots][64]: the sweep after which each vector went quiet (0: not yet)
    unsigned long long* vupd = nullptr; unsigned long long* vdone = nullptr;
    fj_solve_stats* stats = nullptr;
    fj_metrics_out* mets = nullptr;
    int64_t* metric_slot = nullptr;
    std::vector<int64_t> h_metric_slot;
    int64_t total_k = 0;
    int num_colours = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_nodes = 0;
    std::vector<double> tune_ms;
    // launch parameters (set by the tuner): 64-arc chunks in flight per light
    // tile of the union, arcs in flight per lane of the multi-vector rows
    int nch = 4, mu = 8;
    int cache_hit = 0;
    // caller-bound inputs and outputs (fj_batch_bind)
    bool bound = false;
    fj_batch_copy* d_copy_in = nullptr;
    fj_batch_copy* d_copy_out = nullptr;
    int64_t max_item_elems = 0;
    int swept = 0;  // sweeps enqueued by the last solve (budget plus continuations)
    int* d_reopen = nullptr;
    ~fj_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace fj {
namespace {

struct BatchLayoutSizes {
    size_t bytes = 0;
};

// Carve (or size, when base is null) the whole batch workspace.
size_t carve_batch(fj_batch* b, const fj_batch_item_desc* items, int32_t num, void* base) {
    Carver cv(base);
    int64_t un = 0, unnz = 0, ncomp = 0, total_k = 0;
    bool uw = false, udir = false;
    for (int i = 0; i < num; ++i) {
        total_k += items[i].k;
        if (items[i].k == 1) {
            un += items[i].graph.n;
            unnz += items[i].graph.nnz;
            uw = uw || items[i].graph.w != nullptr;
            udir = udir || items[i].graph.directed;
            ++ncomp;
        }
    }
    const int nm = static_cast<int>(num - ncomp);
    const int nslots = static_cast<int>(ncomp) + nm;
    double* somega = cv.take<double>(nslots + 1);
    int* upd = cv.take<int>(nslots + 1);
    int* done = cv.take<int>(nslots + 1);
    int* swd = cv.take<int>(nslots + 1);
    int* vsw = cv.take<int>(64 * (nslots + 1));  // per slot and vector: the sweep after which it was quiet
    int* alld = cv.take<int>(2);  // per branch: union components, multi-vector items
    int* bad = cv.take<int>(1);
    auto* vupd = cv.take<unsigned long long>(nslots + 1);
    auto* vdone = cv.take<unsigned long long>(nslots + 1);
    fj_solve_stats* stats = cv.take<fj_solve_stats>(num);
    fj_metrics_out* mets = cv.take<fj_metrics_out>(total_k);
    int64_t* mslot = cv.take<int64_t>(num);
    auto* cin = cv.take<fj_batch_copy>(num);
    auto* cout = cv.take<fj_batch_copy>(num);
    int* reopen = cv.take<int>(nslots + 1);
    if (b) {
        b->d_copy_in = cin;
        b->d_copy_out = cout;
        b->d_reopen = reopen;
        b->nslots = nslots;
        b->d_slot_omega = somega;
        b->upd = upd; b->done = done; b->sweeps_done = swd; b->all_done = alld; b->bad = bad; b->vsw = vsw;
        b->vupd = vupd; b->vdone = vdone;
        b->stats = stats; b->mets = mets; b->metric_slot = mslot; b->total_k = total_k;
    }
    if (ncomp > 0) {
        UnionGroup* U = b ? &b->U : nullptr;
        auto* rp = cv.take<int32_t>(un + 1);
        auto* col = cv.take<int32_t>(unnz);
        auto* w = uw ? cv.take<float>(unnz) : nullptr;
        auto* noff = cv.take<int64_t>(ncomp + 1);
        auto* citem = cv.take<int32_t>(ncomp);
        auto* cdir = cv.take<int32_t>(ncomp);
        auto* cof = cv.take<int32_t>(un);
        auto* pcomp = cv.take<int32_t>(un);
        fj_graph_desc ud{un, unnz, rp, col, w, 1};
        if (!base) { ud.row_ptr = reinterpret_cast<const int32_t*>(256); ud.col = ud.row_ptr; if (uw) ud.w = reinterpret_cast<const float*>(256); }
        size_t gb = graph_ws_bytes(&ud, FJ_GRAPH_COLOUR | kGraphNoBoundCsr);
        void* gws = cv.take<char>(gb);
        auto* s_in = cv.take<double>(un);
        auto* z_out = cv.take<double>(un);
        auto* sp = cv.take<double>(un);
        auto* zh = cv.take<double>(un);
        auto* zq = cv.take<int32_t>(un);
        auto* partial = cv.take<double>(2 * (unnz / kArcBudget) + 4);
        const int64_t uhc = unnz / kArcBudget + 2;  // heavy rows have more than kArcBudget arcs
        auto* uhcnt = cv.take<int32_t>(uhc);
        auto* ratio = cv.take<double>(un);
        auto* drow = cv.take<double>(un);
        auto* seg = cv.take<double>(8 * ncomp);
        if (U) {
            U->ncomp = static_cast<int>(ncomp); U->n = un; U->nnz = unnz; U->weighted = uw;
            U->row_ptr = rp; U->col = col; U->w = w; U->d_node_off = noff; U->d_comp_item = citem;
            U->comp_dir = cdir; U->comp_of = cof; U->pcomp = pcomp; U->gws = gws; U->gws_bytes = gb;
            U->s_in = s_in; U->z_out = z_out; U->sp = sp; U->zh = zh; U->zq = zq; U->partial = partial;
            U->hcnt = uhcnt; U->hcnt_len = uhc;
            U->ratio = ratio; U->drow = drow; U->seg = seg;
        }
    }
    int mi = 0;
    for (int i = 0; i < num; ++i) {
        if (items[i].k == 1) continue;
        const int64_t n = items[i].graph.n, nnz = items[i].graph.nnz;
        const int k = items[i].k;
        fj_graph_desc d = items[i].graph;
        size_t gb = graph_ws_bytes(&d, FJ_GRAPH_COLOUR | kGraphNoBoundCsr);
        void* gws = cv.take<char>(gb);
        auto* s_in = cv.take<double>(n * k);
        auto* z_out = cv.take<double>(n * k);
        auto* sp = cv.take<double>(n * k);
        auto* zh = cv.take<double>(n * k);
        auto* partial = cv.take<double>((2 * (nnz / kArcBudget) + 4) * k);
        const int64_t mhc = nnz / kArcBudget + 2;
        auto* mhcnt = cv.take<int32_t>(mhc);
        auto* part = cv.take<double>(static_cast<int64_t>(kMBlocks) * 64 * 6);
        auto* tot = cv.take<double>(8 * 64);
        auto* means = cv.take<double>(64);
        if (b) {
            MrhsGroup& G = b->M[mi];
            G.item = i; G.k = k; G.desc = d; G.gws = gws; G.gws_bytes = gb; G.s_in = s_in; G.z_out = z_out;
            G.sp = sp; G.zh = zh; G.partial = partial; G.part = part; G.tot = tot; G.means = means;
            G.hcnt = mhcnt; G.hcnt_len = mhc;
        }
        ++mi;
    }
    return cv.bytes();
}

// the caller-bound copies of every item (inputs before, outputs after a solve)
void enqueue_bound_copy(fj_batch* b, hipStream_t st, const fj_batch_copy* tab) {
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(g1d(b->max_item_elems, 256), 1024));
    hipLaunchKernelGGL(k_batch_copy, dim3(static_cast<unsigned>(per), static_cast<unsigned>(b->num_items)), dim3(256),
                       0, st, tab);
}

// A second stream and two events that let the union and the multi-vector
// branch of a solve run concurrently (used while recording the graph).
struct BranchFork {
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

// Enqueue a batched solve (capture-safe: kernels only): with `init`, the
// start (flags, shift, zero estimate) and sweeps [0, budget); without it,
// sweeps [first, first + budget) continuing from the state in place (slots
// reopened by k_reopen).  Then the results of every item.  With `fork`, the
// multi-vector branch goes to fork->side between a fork and a join on `st`.
fj_status enqueue_solve(fj_batch* b, hipStream_t st, int budget, int* launches_out, int first = 0,
                        bool init = true, const BranchFork* fork = nullptr) {
    int launches = 0;
    const int bs = 256;
    UnionGroup& U = b->U;
    const double epsp = b->epsp;
    SorState SU{U.sp, U.g.popd, U.g.pinv64, U.zh, U.zq, b->omega, 1.0 - 1e-6, epsp, nullptr, nullptr};
    if (init) {
        hipLaunchKernelGGL(k_flags_reset, dim3(1), dim3(256), 0, st, b->nslots, b->upd, b->done, b->sweeps_done,
                           b->all_done, b->bad, b->vupd, b->vdone, b->vsw);
        ++launches;
        if (b->bound) {
            enqueue_bound_copy(b, st, b->d_copy_in);
            ++launches;
        }
        if (b->has_union && U.n > 0) {
            hipLaunchKernelGGL(k_fill_i32, dim3(std::min<int64_t>(g1d(U.hcnt_len, bs), 1024)), dim3(bs), 0, st,
                               U.hcnt_len, U.hcnt, 0);
            ++launches;
            hipLaunchKernelGGL(k_sor_init, dim3(g1d(U.n, bs)), dim3(bs), 0, st, U.n, U.g.perm, U.s_in,
                               static_cast<const double*>(nullptr), b->c, U.sp, U.zh, U.zq, b->bad,
                               static_cast<unsigned long long*>(nullptr));
            ++launches;
        }
        for (auto& G : b->M) {
            hipLaunchKernelGGL(k_fill_i32, dim3(std::min<int64_t>(g1d(G.hcnt_len, bs), 1024)), dim3(bs), 0, st,
                               G.hcnt_len, G.hcnt, 0);
            hipLaunchKernelGGL(k_minit, dim3(g1d(G.g.n * G.k, bs)), dim3(bs), 0, st, G.g.n, G.k, G.g.perm, G.s_in,
                               b->c, G.sp, G.zh, b->bad);
            launches += 2;
        }
    }
    const int last = first + budget;
    // The union's components and the multi-vector items are independent
    // systems: each branch sweeps its own classes and keeps its own sweep
    // bookkeeping, so with a side stream the two run concurrently (a fork
    // before the sweeps, a join after the results); otherwise one after the
    // other on `st`.  Either way every item's arithmetic is the same.
    auto union_branch = [&](hipStream_t bs_st) {
        if (!b->has_union) return;
        for (int sw = first; sw < last; ++sw) {
            for (int k = 0; k < U.g.num_colours; ++k) {
                TileView tv = tile_view(U.g.tiles_p, k);
                if (tv.ntiles + tv.nchunks > 0) {
                    auto kern = b->nch == 2 ? k_usor_tiles<2> : b->nch == 8 ? k_usor_tiles<8> : k_usor_tiles<4>;
                    hipLaunchKernelGGL(kern, dim3(waves_to_blocks(tv.nchunks + tv.ntiles)), dim3(kBlock), 0,
                                       bs_st, tv, U.g.prow_ptr, U.g.pcol, U.g.pw, SU, U.partial, U.hcnt, U.pcomp,
                                       b->d_slot_omega, b->upd, b->done, b->all_done, b->bad);
                    ++launches;
                }
            }
            hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(256), 0, bs_st, 0, U.ncomp, sw, b->upd, b->done,
                               b->sweeps_done, b->all_done, b->vupd, b->vdone, b->vsw);
            ++launches;
        }
        if (U.n == 0) return;
        hipLaunchKernelGGL(k_sor_unshift, dim3(g1d(U.n, bs)), dim3(bs), 0, bs_st, U.n, U.g.perm, U.zh, b->c, U.z_out,
                           static_cast<double*>(nullptr));
        TileView ta = tile_view_all(U.g.tiles_a);
        const unsigned nb1 = waves_to_blocks(ta.nchunks + ta.ntiles), nb2 = waves_to_blocks(ta.h1 - ta.h0);
        hipLaunchKernelGGL(k_urows_tiles<0>, dim3(nb1), dim3(kBlock), 0, bs_st, ta, U.row_ptr, U.col, U.w, U.s_in,
                           U.z_out, U.g.opd, b->c, epsp, U.partial, U.ratio);
        if (nb2) hipLaunchKernelGGL(k_urows_heavy<0>, dim3(nb2), dim3(kBlock), 0, bs_st, ta, U.s_in, U.z_out,
                                    U.g.opd, b->c, epsp, U.partial, U.ratio);
        hipLaunchKernelGGL(k_urows_tiles<1>, dim3(nb1), dim3(kBlock), 0, bs_st, ta, U.row_ptr, U.col, U.w, U.s_in,
                           U.z_out, U.g.opd, b->c, epsp, U.partial, U.drow);
        if (nb2) hipLaunchKernelGGL(k_urows_heavy<1>, dim3(nb2), dim3(kBlock), 0, bs_st, ta, U.s_in, U.z_out,
                                    U.g.opd, b->c, epsp, U.partial, U.drow);
        hipLaunchKernelGGL(k_useg, dim3(U.ncomp), dim3(256), 0, bs_st, U.d_node_off, U.s_in, U.z_out, U.drow, U.ratio,
                           U.seg, 0);
        hipLaunchKernelGGL(k_useg, dim3(U.ncomp), dim3(256), 0, bs_st, U.d_node_off, U.s_in, U.z_out, U.drow, U.ratio,
                           U.seg, 1);
        hipLaunchKernelGGL(k_ufinish, dim3(g1d(U.ncomp, 256)), dim3(256), 0, bs_st, U.ncomp, U.d_comp_item,
                           U.comp_dir, U.d_node_off, U.row_ptr, b->metric_slot, U.seg, b->sweeps_done, 0, last,
                           b->stats, b->mets);
        launches += 7 + (nb2 ? 2 : 0);
    };
    auto multi_branch = [&](hipStream_t bs_st) {
        if (b->M.empty()) return;
        int max_cls = 0;
        for (auto& G : b->M) max_cls = std::max(max_cls, G.g.num_colours);
        for (int sw = first; sw < last; ++sw) {
            for (int k = 0; k < max_cls; ++k) {
                for (size_t m = 0; m < b->M.size(); ++m) {
                    MrhsGroup& G = b->M[m];
                    if (k >= G.g.num_colours) continue;
                    const int slot = U.ncomp + static_cast<int>(m);
                    MState S{G.sp, G.g.popd, G.g.pinv64, G.zh, b->slot_omega[slot], 1.0 - 1e-6, epsp, G.k,
                             b->vdone + slot, b->vupd + slot};
                    TileView tv = tile_view(G.g.tiles_p, k);
                    const int64_t rb = G.g.class_off[k], re = G.g.class_off[k + 1];
                    auto kern = b->mu == 4 ? k_msor_class<4> : b->mu == 16 ? k_msor_class<16> : k_msor_class<8>;
                    hipLaunchKernelGGL(kern, dim3(waves_to_blocks(tv.nchunks + (re - rb))), dim3(kBlock), 0, bs_st,
                                       tv, rb, re, G.g.prow_ptr, G.g.pcol, G.g.pw, S, G.partial, G.hcnt,
                                       b->upd + slot, b->done + slot, b->all_done + 1, b->bad);
                    ++launches;
                }
            }
            hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(256), 0, bs_st, U.ncomp, b->nslots, sw, b->upd, b->done,
                               b->sweeps_done, b->all_done + 1, b->vupd, b->vdone, b->vsw);
            ++launches;
        }
        for (size_t m = 0; m < b->M.size(); ++m) {
            MrhsGroup& G = b->M[m];
            const int slot = U.ncomp + static_cast<int>(m);
            hipLaunchKernelGGL(k_munshift, dim3(g1d(G.g.n * G.k, bs)), dim3(bs), 0, bs_st, G.g.n, G.k, G.g.perm, G.zh,
                               b->c, G.z_out);
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_mresults, dim3(kMBlocks), dim3(kBlock), 0, bs_st, G.g.n, G.k, G.desc.row_ptr,
                                   G.desc.col, G.desc.w, G.g.opd, G.s_in, G.z_out, b->c, epsp, G.means, G.part, pass);
                hipLaunchKernelGGL(k_mreduce, dim3(1), dim3(64), 0, bs_st, G.k, kMBlocks, G.part, G.tot, G.means,
                                   G.g.n, pass);
            }
            hipLaunchKernelGGL(k_mfinish, dim3(1), dim3(64), 0, bs_st, G.k, G.item, G.desc.directed, G.g.n, G.g.nnz,
                               b->h_metric_slot[G.item], G.tot, b->sweeps_done, b->vsw, slot, last, b->stats,
                               b->mets);
            launches += 6;
        }
    };
    if (fork && b->has_union && !b->M.empty()) {
        FJ_HIP(hipEventRecord(fork->ev_fork, st));
        FJ_HIP(hipStreamWaitEvent(fork->side, fork->ev_fork, 0));
        union_branch(st);
        multi_branch(fork->side);
        FJ_HIP(hipEventRecord(fork->ev_join, fork->side));
        FJ_HIP(hipStreamWaitEvent(st, fork->ev_join, 0));
    } else {
        union_branch(st);
        multi_branch(st);
    }
    if (b->bound) {
        enqueue_bound_copy(b, st, b->d_copy_out);
        ++launches;
    }
    b->swept = last;
    if (launches_out) *launches_out = launches;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "enqueue batched solve");
    return FJ_OK;
}

fj_status upload_omegas(fj_batch* b, hipStream_t st) {
    FJ_HIP(hipMemcpyAsync(b->d_slot_omega, b->slot_omega.data(), sizeof(double) * b->nslots, hipMemcpyHostToDevice,
                          st));
    FJ_HIP(hipStreamSynchronize(st));
    return FJ_OK;
}

bool valid_items(const fj_batch_item_desc* items, int32_t num) {
    if (!items || num <= 0) return false;
    for (int i = 0; i < num; ++i) {
        const fj_graph_desc& d = items[i].graph;
        if (items[i].k < 1 || items[i].k > 64) return false;
        if (d.n <= 0 || d.nnz < 0 || !d.row_ptr || (d.nnz > 0 && !d.col)) return false;
        if (d.n >= (int64_t(1) << 31) - 1 || d.nnz >= (int64_t(1) << 31) - 1) return false;
    }
    return true;
}

}  // namespace
}  // namespace fj

extern "C" size_t fj_batch_workspace_bytes(const fj_batch_item_desc* items, int32_t num_items) {
    if (!valid_items(items, num_items)) return 0;
    int64_t un = 0, unnz = 0;
    for (int i = 0; i < num_items; ++i)
        if (items[i].k == 1) { un += items[i].graph.n; unnz += items[i].graph.nnz; }
    if (un >= (int64_t(1) << 31) - 1 || unnz >= (int64_t(1) << 31) - 1) return 0;
    return carve_batch(nullptr, items, num_items, nullptr);
}

extern "C" fj_status fj_batch_create(const fj_batch_item_desc* items, int32_t num_items, const fj_solve_opts* o,
                                     void* ws, size_t ws_bytes, void* stream, fj_batch** out) {
    if (!out || !o || !ws) {
        set_error("fj_batch_create: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!valid_items(items, num_items)) {
        set_error("fj_batch_create: need 1..64 vectors per item and valid graph descriptors");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (!(o->eps > 0.0 && o->eps < 1.0) || !(o->omega > 0.0 && o->omega < 2.0) || !(o->c >= 0.0) ||
        !(o->sigma > 0.0)) {
        set_error("fj_batch_create: need eps in (0,1), omega in (0,2), c >= 0, sigma > 0");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    const size_t need = fj_batch_workspace_bytes(items, num_items);
    if (need == 0 || ws_bytes < need || reinterpret_cast<uintptr_t>(ws) % 256) {
        set_error("fj_batch_create: workspace too small or misaligned (need " + std::to_string(need) + " bytes)");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    fj_batch* b = new (std::nothrow) fj_batch();
    if (!b) {
        set_error("fj_batch_create: host allocation failed");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    b->num_items = num_items;
    b->eps = o->eps; b->omega = o->omega; b->c = o->c; b->sigma = o->sigma;
    b->epsp = o->sigma * o->eps / (o->c + o->sigma);
    int nm = 0;
    for (int i = 0; i < num_items; ++i) {
        b->ks.push_back(items[i].k);
        b->ns.push_back(items[i].graph.n);
        if (items[i].k > 1) ++nm;
    }
    b->M.resize(nm);
    carve_batch(b, items, num_items, ws);
    auto fail = [&](fj_status rc) { delete b; return rc; };
    // metric slots
    b->h_metric_slot.resize(num_items);
    int64_t acc = 0;
    for (int i = 0; i < num_items; ++i) { b->h_metric_slot[i] = acc; acc += items[i].k; }
    if (hipMemcpyAsync(b->metric_slot, b->h_metric_slot.data(), sizeof(int64_t) * num_items, hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return fail(hip_fail(hipGetLastError(), "metric slots"));
    // union of the single-vector items
    UnionGroup& U = b->U;
    if (U.ncomp > 0) {
        b->has_union = true;
        U.node_off.assign(1, 0);
        U.arc_off.assign(1, 0);
        std::vector<int32_t> cdir;
        int* err = b->bad;
        if (hipMemsetAsync(err, 0, sizeof(int), st) != hipSuccess) return fail(hip_fail(hipGetLastError(), "memset"));
        int cidx = 0;
        for (int i = 0; i < num_items; ++i) {
            if (items[i].k != 1) continue;
            const fj_graph_desc& d = items[i].graph;
            U.comp_item.push_back(i);
            cdir.push_back(d.directed ? 1 : 0);
            hipLaunchKernelGGL(k_item_rowptr_check, dim3(g1d(d.n + 1, 256)), dim3(256), 0, st, d.n, d.nnz, d.row_ptr,
                               err);
            int herr = 0;
            if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return fail(hip_fail(hipGetLastError(), "row_ptr check"));
            if (herr) {
                set_error("fj_batch_create: item " + std::to_string(i) + " has an invalid row_ptr");
                return fail(FJ_ERR_INVALID_ARGUMENT);
            }
            hipLaunchKernelGGL(k_union_copy, dim3(g1d(d.n, 256)), dim3(256), 0, st, d.n, d.row_ptr, d.col, d.w,
                               U.node_off.back(), U.arc_off.back(), cidx, U.row_ptr, U.col, U.w, U.comp_of, err);
            U.node_off.push_back(U.node_off.back() + d.n);
            U.arc_off.push_back(U.arc_off.back() + d.nnz);
            ++cidx;
        }
        const int32_t total = static_cast<int32_t>(U.nnz);
        FJ_HIP(hipMemcpyAsync(U.row_ptr + U.n, &total, sizeof(int32_t), hipMemcpyHostToDevice, st));
        FJ_HIP(hipMemcpyAsync(U.d_node_off, U.node_off.data(), sizeof(int64_t) * (U.ncomp + 1), hipMemcpyHostToDevice, st));
        FJ_HIP(hipMemcpyAsync(U.d_comp_item, U.comp_item.data(), sizeof(int32_t) * U.ncomp, hipMemcpyHostToDevice, st));
        FJ_HIP(hipMemcpyAsync(U.comp_dir, cdir.data(), sizeof(int32_t) * U.ncomp, hipMemcpyHostToDevice, st));
        int herr = 0;
        FJ_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
        if (herr) {
            set_error("fj_batch_create: a column index leaves its own graph");
            return fail(FJ_ERR_INVALID_ARGUMENT);
        }
        fj_graph_desc ud{U.n, U.nnz, U.row_ptr, U.col, U.w, 1};
        fj_status rc = graph_build(&U.g, &ud, FJ_GRAPH_COLOUR | kGraphNoBoundCsr, U.gws, U.gws_bytes, st);
        if (rc) return fail(rc);
        hipLaunchKernelGGL(k_union_symmetry, dim3(g1d(U.n, 256)), dim3(256), 0, st, U.n, U.row_ptr, U.col, U.w,
                           U.comp_of, U.comp_dir, err);
        hipLaunchKernelGGL(k_gather_i32, dim3(g1d(U.n, 256)), dim3(256), 0, st, U.n, U.g.perm, U.comp_of, U.pcomp);
        FJ_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
        if (herr) {
            set_error("fj_batch_create: an undirected item is not symmetric");
            return fail(FJ_ERR_INVALID_ARGUMENT);
        }
        b->num_colours = std::max(b->num_colours, U.g.num_colours);
    }
    for (auto& G : b->M) {
        fj_status rc = graph_build(&G.g, &G.desc, FJ_GRAPH_COLOUR | kGraphNoBoundCsr, G.gws, G.gws_bytes, st);
        if (rc) return fail(rc);
        b->num_colours = std::max(b->num_colours, G.g.num_colours);
    }
    b->budget = 256;
    b->slot_omega.assign(b->nslots, b->omega);
    {
        fj_status rc = upload_omegas(b, st);
        if (rc) return fail(rc);
    }
    *out = b;
    return FJ_OK;
}

extern "C" fj_status fj_batch_destroy(fj_batch* b) {
    delete b;
    return FJ_OK;
}

extern "C" fj_status fj_batch_io(const fj_batch* b, int32_t item, double** s, double** z) {
    if (!b || !s || !z || item < 0 || item >= b->num_items) {
        set_error("fj_batch_io: bad argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (b->ks[item] == 1) {
        int cidx = -1;
        for (int q = 0; q < b->U.ncomp; ++q)
            if (b->U.comp_item[q] == item) { cidx = q; break; }
        *s = b->U.s_in + b->U.node_off[cidx];
        *z = b->U.z_out + b->U.node_off[cidx];
    } else {
        for (const auto& G : b->M)
            if (G.item == item) { *s = G.s_in; *z = G.z_out; }
    }
    return FJ_OK;
}

extern "C" fj_status fj_batch_get_info(const fj_batch* b, fj_batch_info* out) {
    if (!b || !out) {
        set_error("fj_batch_get_info: null argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    std::memset(out, 0, sizeof(*out));
    out->omega = b->omega;
    std::vector<int32_t> cdir(b->U.ncomp);
    if (b->U.ncomp) FJ_HIP(hipMemcpy(cdir.data(), b->U.comp_dir, sizeof(int32_t) * b->U.ncomp, hipMemcpyDeviceToHost));
    for (int sl = 0; sl < b->U.ncomp; ++sl) {
        if (cdir[sl]) out->omega_directed = b->slot_omega[sl];
        else out->omega_undirected = b->slot_omega[sl];
    }
    if (!b->M.empty()) out->omega_multi = b->slot_omega[b->U.ncomp];
    out->sweep_budget = b->budget;
    out->graph_nodes = b->graph_nodes;
    out->num_colours = b->num_colours;
    for (size_t i = 0; i < b->tune_ms.size() && i < 16; ++i) out->tune_ms[i] = b->tune_ms[i];
    out->union_chunks_in_flight = b->nch;
    out->multi_arcs_in_flight = b->mu;
    out->cache_hit = b->cache_hit;
    out->bound = b->bound ? 1 : 0;
    return FJ_OK;
}

namespace {

// Record the launch sequence of one solve at the current budget on a private
// stream (the caller's may be the null stream, which cannot be captured);
// fj_solve_batched replays it on the caller's stream.
fj_status record_graph(fj_batch* b) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->graph_nodes = 0;
    hipStream_t cap = nullptr;
    BranchFork fork;
    auto release = [&]() {
        if (cap) (void)hipStreamDestroy(cap);
        if (fork.side) (void)hipStreamDestroy(fork.side);
        if (fork.ev_fork) (void)hipEventDestroy(fork.ev_fork);
        if (fork.ev_join) (void)hipEventDestroy(fork.ev_join);
    };
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&fork.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork.ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork.ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "recording the batch graph");
    }
    int launches = 0;
    fj_status rc = enqueue_solve(b, cap, b->budget, &launches, 0, true, b->concurrent ? &fork : nullptr);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    release();
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    FJ_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_nodes = launches;
    return FJ_OK;
}

// Tuned settings per batch shape, kept for the life of the process: a batch
// whose items fall in the same classes (per item group: count, and the
// base-2 magnitude of nodes and arcs; per multi-vector item: k, nodes, arcs,
// direction; eps, c, sigma) starts from them instead of timing candidates.
struct TunedEntry {
    std::vector<double> slot_omega;
    int nch = 4, mu = 8;
};
std::mutex g_tune_mu;
std::map<std::string, TunedEntry> g_tune_cache;

int log2_bucket(int64_t x) {
    int b = 0;
    while (x > 1) { x >>= 1; ++b; }
    return b;
}

std::string shape_key(const fj_batch* b, const std::vector<int32_t>& cdir) {
    std::string k;
    char buf[160];
    std::snprintf(buf, sizeof(buf), "eps=%.6g c=%.6g sigma=%.6g|", b->eps, b->c, b->sigma);
    k += buf;
    if (b->has_union) {
        int nd = 0;
        for (int32_t d : cdir) nd += d ? 1 : 0;
        std::snprintf(buf, sizeof(buf), "U%d/%d n%d m%d|", b->U.ncomp, nd, log2_bucket(b->U.n), log2_bucket(b->U.nnz));
        k += buf;
    }
    for (const auto& G : b->M) {
        std::snprintf(buf, sizeof(buf), "M k%d n%d m%d d%d|", G.k, log2_bucket(G.g.n), log2_bucket(G.g.nnz),
                      G.desc.directed ? 1 : 0);
        k += buf;
    }
    return k;
}

// Time one solve at the current settings and budget (host clock around a
// synchronized enqueue).
fj_status time_solve(fj_batch* b, hipStream_t st, int budget, double* ms) {
    FJ_HIP(hipStreamSynchronize(st));
    auto t0 = std::chrono::steady_clock::now();
    fj_status rc = enqueue_solve(b, st, budget, nullptr);
    if (rc) return rc;
    FJ_HIP(hipStreamSynchronize(st));
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return FJ_OK;
}

// Sweeps needed per slot at the current settings (0: not within `budget`).
fj_status probe_sweeps(fj_batch* b, hipStream_t st, int budget, std::vector<int>* sweeps, double* ms) {
    fj_status rc = time_solve(b, st, budget, ms);
    if (rc) return rc;
    sweeps->assign(b->nslots, 0);
    FJ_HIP(hipMemcpy(sweeps->data(), b->sweeps_done, sizeof(int) * b->nslots, hipMemcpyDeviceToHost));
    return FJ_OK;
}

}  // namespace

extern "C" void fj_batch_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.clear();
}

extern "C" fj_status fj_batch_tune(fj_batch* b, const double* omegas, int32_t n_omegas, void* stream) {
    if (!b || !omegas || n_omegas < 1 || n_omegas > 16) {
        set_error("fj_batch_tune: need 1..16 candidate omegas");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    for (int q = 0; q < n_omegas; ++q)
        if (!(omegas[q] > 0.0 && omegas[q] < 2.0)) {
            set_error("fj_batch_tune: omega must be in (0,2)");
            return FJ_ERR_INVALID_ARGUMENT;
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->graph_nodes = 0;
    b->tune_ms.assign(n_omegas, 0.0);
    b->cache_hit = 0;
    const int probe_budget = 512;
    std::vector<int32_t> cdir(b->U.ncomp);
    if (b->U.ncomp) FJ_HIP(hipMemcpy(cdir.data(), b->U.comp_dir, sizeof(int32_t) * b->U.ncomp, hipMemcpyDeviceToHost));
    const std::string key = shape_key(b, cdir);
    TunedEntry cached;
    bool hit = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && static_cast<int>(it->second.slot_omega.size()) == b->nslots) {
            cached = it->second;
            hit = true;
        }
    }
    int budget = 0;
    if (hit) {
        // the cached settings; one solve with a generous budget sets the sweep budget for these inputs
        b->slot_omega = cached.slot_omega;
        b->nch = cached.nch;
        b->mu = cached.mu;
        fj_status rc = upload_omegas(b, st);
        if (rc) return rc;
        std::vector<int> sw;
        double ms = 0.0;
        rc = probe_sweeps(b, st, probe_budget, &sw, &ms);
        if (rc) return rc;
        for (int sl = 0; sl < b->nslots; ++sl) {
            if (sw[sl] == 0) { hit = false; break; }
            budget = std::max(budget, sw[sl]);
        }
        b->cache_hit = hit ? 1 : 0;
    }
    if (!hit) {
        b->nch = 4;
        b->mu = 8;
        // sweeps[q][slot]: sweeps slot needed with candidate q (0: did not converge)
        std::vector<std::vector<int>> sweeps(n_omegas);
        for (int q = 0; q < n_omegas; ++q) {
            b->slot_omega.assign(b->nslots, omegas[q]);
            fj_status rc = upload_omegas(b, st);
            if (rc) return rc;
            rc = probe_sweeps(b, st, probe_budget, &sweeps[q], &b->tune_ms[q]);
            if (rc) return rc;
        }
        // One omega per group: the multi-vector items one each, the undirected and
        // the directed union components one per kind (their launches are shared,
        // so each kind is judged by its slowest component).
        std::vector<int> group(b->nslots);
        for (int sl = 0; sl < b->nslots; ++sl) group[sl] = sl < b->U.ncomp ? cdir[sl] : 2 + (sl - b->U.ncomp);
        const int ngroups = 2 + static_cast<int>(b->M.size());
        b->slot_omega.assign(b->nslots, b->omega);
        bool all_ok = true;
        for (int gidx = 0; gidx < ngroups; ++gidx) {
            int best_q = -1, best_sw = 1 << 30;
            bool any = false;
            for (int q = 0; q < n_omegas; ++q) {
                int worst = 0;
                bool ok = true;
                for (int sl = 0; sl < b->nslots; ++sl) {
                    if (group[sl] != gidx) continue;
                    any = true;
                    if (sweeps[q][sl] == 0) ok = false;
                    worst = std::max(worst, sweeps[q][sl]);
                }
                if (ok && worst < best_sw) { best_sw = worst; best_q = q; }
            }
            if (!any) continue;
            if (best_q < 0) { all_ok = false; continue; }
            for (int sl = 0; sl < b->nslots; ++sl)
                if (group[sl] == gidx) b->slot_omega[sl] = omegas[best_q];
            budget = std::max(budget, best_sw);
        }
        if (!all_ok) {
            set_error("fj_batch_tune: some item did not converge within 512 sweeps for any candidate omega");
            return FJ_ERR_NOT_CONVERGED;
        }
        fj_status rc = upload_omegas(b, st);
        if (rc) return rc;
        // Launch parameters at the chosen omegas and budget, one at a time:
        // 64-arc chunks in flight per light tile of the union (2, 4, 8), then
        // arcs in flight per wave of the multi-vector rows (4, 8, 16).  Either
        // leaves the sums, hence the result, unchanged.
        const int run_budget = budget + 1;
        double best_ms = 0.0;
        rc = time_solve(b, st, run_budget, &best_ms);  // nch = 4, mu = 8
        if (rc) return rc;
        const int cand[2] = {2, 8};
        if (b->has_union) {
            int best = 4;
            for (int c : cand) {
                b->nch = c;
                double ms = 0.0;
                rc = time_solve(b, st, run_budget, &ms);
                if (rc) return rc;
                if (ms < 0.98 * best_ms) { best_ms = ms; best = c; }
            }
            b->nch = best;
        }
        if (!b->M.empty()) {
            int best = 8;
            for (int c : {4, 16}) {
                b->mu = c;
                double ms = 0.0;
                rc = time_solve(b, st, run_budget, &ms);
                if (rc) return rc;
                if (ms < 0.98 * best_ms) { best_ms = ms; best = c; }
            }
            b->mu = best;
        }
        TunedEntry e;
        e.slot_omega = b->slot_omega;
        e.nch = b->nch;
        e.mu = b->mu;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = e;
    }
    b->omega = b->slot_omega.empty() ? b->omega : b->slot_omega.back();
    b->budget = budget + std::max(4, budget / 4);
    return record_graph(b);
}

extern "C" fj_status fj_batch_bind(fj_batch* b, const double* const* s, double* const* z, void* stream) {
    if (!b || (!s) != (!z)) {
        set_error("fj_batch_bind: need a batch and both pointer arrays (or neither, to unbind)");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!s) {
        b->bound = false;
    } else {
        std::vector<fj_batch_copy> in(b->num_items), out(b->num_items);
        int64_t mx = 0;
        for (int i = 0; i < b->num_items; ++i) {
            if (!s[i] || !z[i] || reinterpret_cast<uintptr_t>(s[i]) % 8 || reinterpret_cast<uintptr_t>(z[i]) % 8) {
                set_error("fj_batch_bind: item " + std::to_string(i) + " has a null or misaligned pointer");
                return FJ_ERR_INVALID_ARGUMENT;
            }
            double *si = nullptr, *zi = nullptr;
            fj_status rc = fj_batch_io(b, i, &si, &zi);
            if (rc) return rc;
            const int64_t cnt = b->ns[i] * b->ks[i];
            in[i] = fj_batch_copy{s[i], si, cnt};
            out[i] = fj_batch_copy{zi, z[i], cnt};
            mx = std::max(mx, cnt);
        }
        FJ_HIP(hipMemcpyAsync(b->d_copy_in, in.data(), sizeof(fj_batch_copy) * b->num_items, hipMemcpyHostToDevice, st));
        FJ_HIP(hipMemcpyAsync(b->d_copy_out, out.data(), sizeof(fj_batch_copy) * b->num_items, hipMemcpyHostToDevice,
                              st));
        FJ_HIP(hipStreamSynchronize(st));
        b->max_item_elems = mx;
        b->bound = true;
    }
    // a recorded graph holds the copies or not: record it again at the same settings
    if (b->exec) return record_graph(b);
    return FJ_OK;
}

extern "C" fj_status fj_batch_check(fj_batch* b, int32_t extra_sweeps, int32_t* uncertified,
                                    fj_solve_stats* stats_dev, fj_metrics_out* metrics_dev, void* stream) {
    if (!b || !uncertified || extra_sweeps < 0 || extra_sweeps > 100000) {
        set_error("fj_batch_check: bad argument");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<fj_solve_stats> hs(b->num_items);
    auto count = [&](std::vector<int>* open) -> fj_status {
        FJ_HIP(hipMemcpyAsync(hs.data(), b->stats, sizeof(fj_solve_stats) * b->num_items, hipMemcpyDeviceToHost, st));
        FJ_HIP(hipStreamSynchronize(st));
        int c = 0;
        if (open) open->clear();
        for (int i = 0; i < b->num_items; ++i) {
            if (hs[i].certified) continue;
            ++c;
            if (!open) continue;
            if (b->ks[i] == 1) {
                for (int q = 0; q < b->U.ncomp; ++q)
                    if (b->U.comp_item[q] == i) open->push_back(q);
            } else {
                for (size_t m = 0; m < b->M.size(); ++m)
                    if (b->M[m].item == i) open->push_back(b->U.ncomp + static_cast<int>(m));
            }
        }
        *uncertified = c;
        return FJ_OK;
    };
    std::vector<int> open;
    fj_status rc = count(&open);
    if (rc) return rc;
    if (*uncertified > 0 && extra_sweeps > 0) {
        // Lemma 4: the estimates in place are a valid start; the reopened
        // items sweep on from them to the same certificate
        const int first = b->swept;
        FJ_HIP(hipMemcpyAsync(b->d_reopen, open.data(), sizeof(int) * open.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_reopen, dim3(1), dim3(256), 0, st, static_cast<int>(open.size()), b->d_reopen, b->done,
                           b->sweeps_done, b->all_done, b->vdone);
        rc = enqueue_solve(b, st, extra_sweeps, nullptr, first, false);
        if (rc) return rc;
        rc = count(nullptr);
        if (rc) return rc;
    }
    if (stats_dev)
        FJ_HIP(hipMemcpyAsync(stats_dev, b->stats, sizeof(fj_solve_stats) * b->num_items, hipMemcpyDeviceToDevice, st));
    if (metrics_dev)
        FJ_HIP(hipMemcpyAsync(metrics_dev, b->mets, sizeof(fj_metrics_out) * b->total_k, hipMemcpyDeviceToDevice, st));
    if (stats_dev || metrics_dev) FJ_HIP(hipStreamSynchronize(st));
    if (*uncertified > 0) {
        set_error("fj_batch_check: " + std::to_string(*uncertified) + " item(s) not certified");
        return FJ_ERR_NOT_CONVERGED;
    }
    return FJ_OK;
}

extern "C" fj_status fj_solve_batched(fj_batch* b, fj_solve_stats* stats_dev, fj_metrics_out* metrics_dev,
                                      void* stream) {
    if (!b) {
        set_error("fj_solve_batched: null batch");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (b->exec) {
        FJ_HIP(hipGraphLaunch(b->exec, st));
        b->swept = b->budget;
    } else {
        fj_status rc = enqueue_solve(b, st, b->budget, nullptr);
        if (rc) return rc;
    }
    if (stats_dev)
        FJ_HIP(hipMemcpyAsync(stats_dev, b->stats, sizeof(fj_solve_stats) * b->num_items, hipMemcpyDeviceToDevice, st));
    if (metrics_dev)
        FJ_HIP(hipMemcpyAsync(metrics_dev, b->mets, sizeof(fj_metrics_out) * b->total_k, hipMemcpyDeviceToDevice, st));
    return FJ_OK;
}

extern "C" fj_status fj_batch_set_launch(fj_batch* b, int32_t union_chunks, int32_t multi_arcs) {
    const bool ok_u = union_chunks == 0 || union_chunks == 2 || union_chunks == 4 || union_chunks == 8;
    const bool ok_m = multi_arcs == 0 || multi_arcs == 4 || multi_arcs == 8 || multi_arcs == 16;
    if (!b || !ok_u || !ok_m) {
        set_error("fj_batch_set_launch: need a batch, union_chunks in {0, 2, 4, 8} and multi_arcs in {0, 4, 8, 16}");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (union_chunks) b->nch = union_chunks;
    if (multi_arcs) b->mu = multi_arcs;
    return b->exec ? record_graph(b) : FJ_OK;
}

extern "C" fj_status fj_batch_set_omegas(fj_batch* b, double omega_undirected, double omega_directed,
                                         double omega_multi) {
    if (!b || omega_undirected >= 2.0 || omega_directed >= 2.0 || omega_multi >= 2.0) {
        set_error("fj_batch_set_omegas: need a batch and omegas below 2");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    std::vector<int32_t> cdir(b->U.ncomp);
    if (b->U.ncomp) FJ_HIP(hipMemcpy(cdir.data(), b->U.comp_dir, sizeof(int32_t) * b->U.ncomp, hipMemcpyDeviceToHost));
    for (int sl = 0; sl < b->nslots; ++sl) {
        double w = sl < b->U.ncomp ? (cdir[sl] ? omega_directed : omega_undirected) : omega_multi;
        if (w > 0.0) b->slot_omega[sl] = w;
    }
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->graph_nodes = 0;
    return upload_omegas(b, nullptr);
}
