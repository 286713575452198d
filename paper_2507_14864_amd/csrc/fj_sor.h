// Colour-ordered over-relaxed sweep kernels shared by the single solve and the
// batched solve.
//
// Relabelled graph: colour class k occupies a contiguous row range.  Rows of
// one class are not adjacent in A + A^T, so updating them together is exactly
// the sequential Gauss-Seidel update of each (Thm. 8), over-relaxed by omega
// (Eq. (sor1)).  Pull form: r_i = s'_i - (1+d_i) zhat'_i + sum_j a_ij zhat'_j
// is recomputed from the current estimate (equal to the tracked residual by
// Lemma 4), and row i is updated iff |r_i| > h_i = eps' s'_i (Alg. 3's test).
#pragma once
#include "fj_device.h"
#include "fj_internal.h"
#include "fj_tile.h"

namespace fj {
namespace {

__device__ __forceinline__ void flag_set(int* f) {
    if (__atomic_load_n(f, __ATOMIC_RELAXED) == 0) __atomic_store_n(f, 1, __ATOMIC_RELAXED);
}
__device__ __forceinline__ void stripe_add(unsigned long long* stats, int slot, unsigned long long v) {
    atomicAdd(&stats[(blockIdx.x % kStripes) * kStripeStride + slot], v);
}

// 32-bit fixed-point copy of zhat' (scale 2^30, range (-2, 2)) used by the
// light-row gathers while the sweeps are far from the certificate: half the
// bytes of FP64 and an absolute resolution of 9.3e-10 (FP32 would give 6e-8
// near 1).  The final sweeps and the certificate read FP64 only.
constexpr double kFixScale = 1073741824.0;  // 2^30
__device__ __forceinline__ int32_t fix_enc(double z) {
    double q = rint(z * kFixScale);
    q = fmin(fmax(q, -2147483647.0), 2147483647.0);
    return static_cast<int32_t>(q);
}
__device__ __forceinline__ double fix_dec(int32_t q) { return static_cast<double>(q) * (1.0 / kFixScale); }

struct SorState {
    const double* sp;    // s' = s + c, relabelled
    const double* popd;  // 1 + d
    const double* pinv;  // 1 / (1 + d)
    double* zh;          // zhat', FP64
    int32_t* zq;         // fixed-point copy of zhat'
    double omega;
    double thr;          // update iff |r| > thr * eps' s'
    double epsp;
    unsigned long long* hacc;             // per heavy row: packed fixed-point sum and chunk count
    const unsigned long long* zmax_bits;  // bits of max |zhat'| at the start (a nonnegative double)
    double* zsh;                          // merged tail: new zhat' of rows >= sh_base (shadow)
    int32_t* zqsh;                        // merged tail: new fixed-point copy (shadow)
    int64_t sh_base;
};

// Grid-stride over the nodes; one atomic per block for the magnitude bound.
__global__ __launch_bounds__(256) void k_sor_init(int64_t n, const int32_t* __restrict__ perm,
                                                  const double* __restrict__ s, const double* __restrict__ z0,
                                                  double c, double* sp, double* zh, int32_t* zq, int* bad,
                                                  unsigned long long* zmax_bits) {
    __shared__ double s_max[4];
    double m = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t o = perm ? perm[i] : i;
        double si = s[o];
        if (!(si >= 0.0) || !isfinite(si)) flag_set(bad);
        sp[i] = si + c;
        double z = 0.0;
        if (z0) {
            double zi = z0[o];
            if (!isfinite(zi)) flag_set(bad);
            z = zi + c;
        }
        zh[i] = z;
        zq[i] = fix_enc(z);
        double mi = fmax(si + c, fabs(z));
        if (isfinite(mi)) m = fmax(m, mi);
    }
    if (!zmax_bits) return;  // uniform
    m = wave_max(m);
    if (lane_id() == 0) s_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (blockDim.x >> 6); ++w) m = fmax(m, s_max[w]);
        // nonnegative doubles order like their bit patterns
        if (m > 0.0) atomicMax(zmax_bits, static_cast<unsigned long long>(__double_as_longlong(m)));
    }
}

// The row's own data is touched once per sweep: streaming (nontemporal) loads
// and stores keep it from displacing the gathered values in L2.
struct RowData {
    double z, sp, opd, inv;
};
// A light row that gathers the copy sees a sum off by at most 2^-31 d_i.
// Where that exceeds the 5% margin the fixed-point sweeps keep below the
// threshold (2^-31 d_i > 0.05 eps' s'_i: large degree, tiny opinion) the row
// gathers FP64 instead, so the fixed-point sweeps can always go quiet.
__device__ __forceinline__ bool fix_too_coarse(const RowData& d, double epsp) {
    return (d.opd - 1.0) * (0.5 / kFixScale) > 0.05 * epsp * d.sp;
}

__device__ __forceinline__ RowData row_load(int64_t i, const SorState& S) {
    return RowData{__builtin_nontemporal_load(&S.zh[i]), __builtin_nontemporal_load(&S.sp[i]),
                   __builtin_nontemporal_load(&S.popd[i]), __builtin_nontemporal_load(&S.pinv[i])};
}
// Test and update with the row's data already loaded (the kernels issue these
// loads before the arc loop, so they are not on the critical path).  In a
// merged tail launch (SHADOW) every row writes its new or unchanged value to
// the shadow arrays, so rows of the launch gather only values from before it.
template <bool SHADOW = false>
__device__ __forceinline__ bool sor_row_with(int64_t i, const RowData& d, double sum, const SorState& S,
                                             bool* nonfinite, double slack = 0.0) {
    const double ri = d.sp - d.opd * d.z + sum;
    *nonfinite = !isfinite(ri);
    const bool upd = fabs(ri) > S.thr * S.epsp * d.sp + slack;
    const double z = upd ? d.z + S.omega * ri * d.inv : d.z;
    if constexpr (SHADOW) {
        S.zsh[i - S.sh_base] = z;
        S.zqsh[i - S.sh_base] = fix_enc(z);
    } else if (upd) {
        __builtin_nontemporal_store(z, &S.zh[i]);
        __builtin_nontemporal_store(fix_enc(z), &S.zq[i]);
    }
    return upd;
}
__device__ __forceinline__ bool sor_row(int64_t i, double sum, const SorState& S, bool* nonfinite) {
    return sor_row_with(i, row_load(i, S), sum, S, nonfinite);
}

// Row sums of a light tile.  FP64 sweeps gather zhat'; fixed-point sweeps
// gather the 32-bit copy, except for rows the copy cannot resolve
// (fix_too_coarse), which gather zhat' (flags in LDS, checked per arc only
// when the tile holds such a row).  rd: the lane's row data (lane < nrows).
template <bool MIRROR>
__device__ __forceinline__ double light_tile_sums(const int32_t* __restrict__ prow_ptr, const int32_t* __restrict__ pcol,
                                                  const float* __restrict__ pw, const SorState& S, int32_t r0,
                                                  int nrows, const RowData& rd, int* pre, double* acc, int* flag) {
    const double* __restrict__ zh = S.zh;
    const int32_t* __restrict__ zq = S.zq;
    const int lane = lane_id();
    auto arc64 = [&](int k) {
        double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
        return a * zh[__builtin_nontemporal_load(&pcol[k])];
    };
    if constexpr (!MIRROR) {
        return tile_row_sums(prow_ptr, r0, nrows, pre, acc, arc64);
    } else {
        auto arcq = [&](int k) {
            double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
            return a * fix_dec(zq[__builtin_nontemporal_load(&pcol[k])]);
        };
        const bool coarse = lane < nrows && fix_too_coarse(rd, S.epsp);
        if (!__ballot(coarse)) return tile_row_sums(prow_ptr, r0, nrows, pre, acc, arcq);
        flag[lane] = coarse ? 1 : 0;  // published by the LDS sync inside tile_row_sums
        return tile_row_sums(prow_ptr, r0, nrows, pre, acc,
                             [&](int k, int slot) { return flag[slot] ? arc64(k) : arcq(k); });
    }
}

template <bool MIRROR>
__global__ __launch_bounds__(kBlock) void k_sor_tiles(TileView tv, const int32_t* __restrict__ prow_ptr,
                                                      const int32_t* __restrict__ pcol, const float* __restrict__ pw,
                                                      SorState S, double* partial, const int* prev, int* updated,
                                                      int* bad, unsigned long long* stats) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    __shared__ int s_flag[kWavesPerBlock][64];
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    const int wid = threadIdx.x >> 6, lane = lane_id();
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    const double* __restrict__ zh = S.zh;
    auto arc64 = [&](int k) {
        double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
        return a * zh[__builtin_nontemporal_load(&pcol[k])];
    };
    if (wv < tv.nchunks) {  // heavy rows always gather FP64
        int64_t cidx = tv.c0 + wv;
        int32_t row = tv.heavy_row[tv.chunk_heavy[cidx]];
        int beg = tv.chunk_beg[cidx];
        int end = min(beg + kArcBudget, prow_ptr[row + 1]);
        double sum = chunk_sum(beg, end, arc64);
        if (lane == 0) partial[cidx] = sum;
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;  // finished by k_sor_heavy
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    RowData rd{};
    if (lane < nrows) rd = row_load(r0 + lane, S);
    const double sum = light_tile_sums<MIRROR>(prow_ptr, pcol, pw, S, r0, nrows, rd, s_pre[wid], s_acc[wid],
                                               s_flag[wid]);
    bool upd = false, nonfinite = false;
    if (lane < nrows) upd = sor_row_with(r0 + lane, rd, sum, S, &nonfinite);
    uint64_t um = __ballot(upd);
    if (__ballot(nonfinite) && lane == 0) flag_set(bad);
    if (um && lane == 0) {
        flag_set(updated);
        stripe_add(stats, 0, static_cast<unsigned long long>(__popcll(um)));
    }
}

// Heavy rows inside one launch.  Every chunk wave converts its FP64 partial
// sum p to the integer P = round(p 2^F) with a per-row F chosen from the row's
// weighted degree d and a bound zb on |zhat'| so that the row's partials have
// sum |P| <= 2^82 (the absolute partials of a row sum to at most d zb).  P is
// split into H = P >> 32 (signed) and L = P mod 2^32, and the wave adds
// (H << 12) + 1 to one 64-bit word of the row and (L << 12) + 1 to the other:
// each word carries its own arrival count in the low 12 bits, and the sums of
// H and of L stay inside the 52 bits above it.  Integer addition is
// associative, so the total does not depend on the order in which chunks
// arrive.  Its resolution, 2^-82 d zb per chunk, lies some 2^29 below the FP64
// rounding of the partial itself.  The two additions are issued back to back;
// the wave that completes the count of the L word owns the total.  If its own
// H addition did not complete the H word it polls that word: every missing H
// addition belongs to a resident wave that has already performed its L
// addition, so it is in flight or next to issue and the poll ends; a bounded
// poll flags the solve as failed rather than wait without end.  The owner updates the row and clears both words for the next
// launch.  A partial outside the range flags the solve as diverged; a row
// total outside it (only if |zhat'| grew past twice zb) yields a wrong sum
// that the final FP64 certificate rejects.
constexpr int kFixBits = 82;
constexpr int kHeavyPoll = 1 << 16;
__device__ __forceinline__ int heavy_frac_bits(double d, const unsigned long long* zmax_bits) {
    const double zb = 4.0 * __longlong_as_double(static_cast<long long>(*zmax_bits));
    const double bound = fmax(d * zb, 1e-300);
    return kFixBits - static_cast<int>(ceil(log2(bound)));
}
// P = round(p 2^F) (halves toward +infinity); false if |P| > 2^kFixBits or p not finite
__device__ __forceinline__ bool to_fixed128(double p, int F, __int128* out) {
    if (!isfinite(p)) return false;
    if (p == 0.0) { *out = 0; return true; }
    int x;
    const double m = frexp(p, &x);  // p = m 2^x, 0.5 <= |m| < 1
    const long long M = static_cast<long long>(ldexp(m, 53));
    const int s = x - 53 + F;
    if (x + F > kFixBits + 1) return false;  // |p| 2^F >= 2^(kFixBits+1)
    __int128 P;
    if (s >= 0) P = static_cast<__int128>(M) << s;
    else if (s <= -64) P = 0;
    else P = (static_cast<__int128>(M) + (static_cast<__int128>(1) << (-s - 1))) >> (-s);
    const __int128 lim = static_cast<__int128>(1) << kFixBits;
    if (P > lim || P < -lim) return false;
    *out = P;
    return true;
}

// One colour class in a single launch: the first nchunks waves each sum one
// heavy-row chunk (combined as above), the rest take one light tile each.
// Used when no heavy row of the class has more than kMaxPackedChunks chunks.
// SHADOW: the launch covers several trailing classes at once (a merged tail);
// rows write to the shadow arrays and k_sor_commit publishes them afterwards,
// so within the launch every gather sees values from before it.
// A sweep that follows a quiet sweep (no row updated) would change nothing:
// when *prev is 0 the launch returns at once.
template <bool MIRROR, bool SHADOW>
__global__ __launch_bounds__(kBlock) void k_sor_class(TileView tv, const int32_t* __restrict__ prow_ptr,
                                                      const int32_t* __restrict__ pcol, const float* __restrict__ pw,
                                                      SorState S, const int* prev, int* updated, int* bad,
                                                      unsigned long long* stats) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    __shared__ int s_flag[kWavesPerBlock][64];
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    const int wid = threadIdx.x >> 6, lane = lane_id();
    const double* __restrict__ zh = S.zh;
    int64_t wv = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (wv < tv.nchunks) {  // heavy rows always gather FP64
        auto arc64 = [&](int k) {
            double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
            return a * zh[__builtin_nontemporal_load(&pcol[k])];
        };
        const int64_t cidx = tv.c0 + wv;
        const int beg = tv.chunk_beg[cidx];
        const int end = tv.chunk_end[cidx];
        const int32_t h = tv.chunk_heavy[cidx];
        // row, chunk count and the row's data load while the arcs stream
        const int32_t row = tv.heavy_row[h];
        const int nch = tv.heavy_chunk0[h + 1] - tv.heavy_chunk0[h];
        RowData rd{};
        if (lane == 0) rd = row_load(row, S);
        const double part = chunk_sum(beg, end, arc64);
        if (lane == 0) {
            const int F = heavy_frac_bits(rd.opd - 1.0, S.zmax_bits);
            __int128 P = 0;
            if (!to_fixed128(part, F, &P)) flag_set(bad);
            constexpr unsigned long long cmask = kMaxPackedChunks;
            const unsigned long long addh =
                (static_cast<unsigned long long>(static_cast<long long>(P >> 32)) << kPackedCountBits) + 1ull;
            const unsigned long long addl =
                (static_cast<unsigned long long>(P & static_cast<__int128>(0xffffffffull)) << kPackedCountBits) + 1ull;
            unsigned long long* acc = S.hacc + 2 * static_cast<int64_t>(h);
            const unsigned long long oldh = atomicAdd(&acc[0], addh);
            const unsigned long long oldl = atomicAdd(&acc[1], addl);
            if (static_cast<int>(oldl & cmask) + 1 == nch) {
                unsigned long long th = oldh + addh;
                for (int poll = 0; static_cast<int>(th & cmask) != nch; ++poll) {
                    if (poll == kHeavyPoll) {
                        flag_set(bad);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    th = atomicAdd(&acc[0], 0ull);
                }
                const unsigned long long tl = oldl + addl;
                atomicExch(&acc[0], 0ull);
                atomicExch(&acc[1], 0ull);
                const double tot = ldexp(static_cast<double>(static_cast<long long>(th) >> kPackedCountBits), 32 - F) +
                                   ldexp(static_cast<double>(tl >> kPackedCountBits), -F);
                bool nonfinite = false;
                bool upd = sor_row_with<SHADOW>(row, rd, tot, S, &nonfinite);
                if (nonfinite) flag_set(bad);
                if (upd) {
                    flag_set(updated);
                    stripe_add(stats, 0, 1ull);
                }
            }
        }
        return;
    }
    wv -= tv.nchunks;
    if (wv >= tv.ntiles) return;
    const int64_t tix = tv.t0 + wv;
    if (tv.tile_heavy[tix] >= 0) return;  // taken by the chunk waves
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    RowData rd{};
    if (lane < nrows) rd = row_load(r0 + lane, S);
    const double sum = light_tile_sums<MIRROR>(prow_ptr, pcol, pw, S, r0, nrows, rd, s_pre[wid], s_acc[wid],
                                               s_flag[wid]);
    bool upd = false, nonfinite = false;
    if (lane < nrows) upd = sor_row_with<SHADOW>(r0 + lane, rd, sum, S, &nonfinite);
    uint64_t um = __ballot(upd);
    if (__ballot(nonfinite) && lane == 0) flag_set(bad);
    if (um && lane == 0) {
        flag_set(updated);
        stripe_add(stats, 0, static_cast<unsigned long long>(__popcll(um)));
    }
}

// after a merged tail launch: the shadow values become the estimate
__global__ void k_sor_commit(int64_t base, int64_t n, const double* __restrict__ zsh, const int32_t* __restrict__ zqsh,
                             double* zh, int32_t* zq, const int* prev) {
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    const int64_t i = base + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    zh[i] = zsh[i - base];
    zq[i] = zqsh[i - base];
}

__global__ __launch_bounds__(kBlock) void k_sor_heavy(TileView tv, SorState S, const double* __restrict__ partial,
                                                      const int* prev, int* updated, int* bad,
                                                      unsigned long long* stats) {
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    const int wid = threadIdx.x >> 6, lane = lane_id();
    int64_t hh = tv.h0 + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wid;
    if (hh >= tv.h1) return;
    int32_t c0 = tv.heavy_chunk0[hh], c1 = tv.heavy_chunk0[hh + 1];
    double sum = 0.0;
    for (int32_t c = c0 + lane; c < c1; c += 64) sum += partial[c];
    sum = wave_sum(sum);
    if (lane == 0) {
        bool nonfinite = false;
        bool upd = sor_row(tv.heavy_row[hh], sum, S, &nonfinite);
        if (nonfinite) flag_set(bad);
        if (upd) {
            flag_set(updated);
            stripe_add(stats, 0, 1ull);
        }
    }
}


__global__ void k_sor_unshift(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ zh, double c,
                              double* z, double* zh_orig) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = perm[i];
    z[o] = zh[i] - c;
    if (zh_orig) zh_orig[o] = zh[i];
}

}  // namespace
}  // namespace fj
