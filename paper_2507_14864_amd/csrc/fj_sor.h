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
    // Bound skipping (k_sor_class).  ub[i] bounds |r_i|
    // for the current estimate: the row's own residual at its last sweep
    // (after its own update, (1 - omega) of it, Eq. (sor2)), plus
    // a_ij |change of zhat'_j| for every neighbour update since (Lemma 4: a
    // change of zhat'_j moves r_i by a_ij times it).  A row whose bound plus
    // its gather error stays below the update threshold would not update, so
    // it keeps its value without gathering: the same iteration, bit for bit.
    // The sweep's mode (k_sweep_begin) is a separate kernel argument.
    double* ub;       // [n]
    double* ub_tail;  // [n - sh_base]: adds made inside a merged-tail launch to
                      // its own rows, merged into ub at the next sweep's start
    // The rows whose bounds an update of row i raises, with the arc weights:
    // the rows j with a_ji > 0, i.e. row i of the relabelled CSR(A^T) (of
    // CSR(A) itself when the pattern is symmetric).
    const int32_t* brow;
    const int32_t* bcol;
    const float* bw;
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
                                             bool* nonfinite, double* r_out = nullptr, double* z_out = nullptr) {
    const double ri = d.sp - d.opd * d.z + sum;
    *nonfinite = !isfinite(ri);
    const bool upd = fabs(ri) > S.thr * S.epsp * d.sp;
    const double z = upd ? d.z + S.omega * ri * d.inv : d.z;
    if (r_out) *r_out = ri;
    if (z_out) *z_out = z;
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
// A skipped row keeps its value; in a merged tail launch it still writes it
// to the shadow arrays, which the commit copies back.
template <bool SHADOW>
__device__ __forceinline__ void keep_row(int64_t i, const RowData& d, const SorState& S) {
    if constexpr (SHADOW) {
        S.zsh[i - S.sh_base] = d.z;
        S.zqsh[i - S.sh_base] = fix_enc(d.z);
    }
}

// Bound skipping.  The residual a sweep computes for row i differs from the
// exact residual of the stored estimate by at most resid_err: the 32-bit copy
// is off by at most 2^-31 per unit of arc weight, and the FP64 sums and the
// update round far below that.
__device__ __forceinline__ double resid_err(double opd) { return opd * 0x1p-30; }
// the bound a row keeps after its own sweep: the exact residual is within
// resid_err of the computed r; an update by omega r / (1 + d) leaves
// (1 - omega) r plus the rounding of the update
__device__ __forceinline__ double own_bound(double r, bool upd, double omega, double opd) {
    const double e = resid_err(opd);
    return upd ? (fabs(1.0 - omega) * fabs(r) + 2.0 * e) * (1.0 + 0x1p-40) : fabs(r) + e;
}
// true when the row provably would not update: its computed residual is at
// most ub + resid_err, below the threshold
__device__ __forceinline__ bool bound_quiet(double ub, const RowData& d, const SorState& S) {
    return ub + resid_err(d.opd) < 0.999 * S.thr * S.epsp * d.sp;
}
// An update of zhat'_i by delta (mag >= |delta|) adds a_ji mag to the bound of
// every row j that reads it (row i of S.brow/S.bcol/S.bw).  The whole wave
// takes the arcs [beg, end) of that row, U loads in flight per lane (the
// atomics return nothing).  Inside a merged-tail launch the tail's own rows
// collect in ub_tail, since they may be computing their bounds concurrently.
template <int U, bool SHADOW>
__device__ __forceinline__ void bound_arcs(const SorState& S, int beg, int end, double mag) {
    const int32_t* __restrict__ pcol = S.bcol;
    const float* __restrict__ pw = S.bw;
    for (int k0 = beg + lane_id(); k0 < end; k0 += 64 * U) {
        int j[U];
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + 64 * u;
            j[u] = k < end ? pcol[k] : -1;
            a[u] = pw && k < end ? static_cast<double>(pw[k]) : 1.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j[u] < 0) continue;
            if (SHADOW && j[u] >= S.sh_base) atomic_add_noret(&S.ub_tail[j[u] - S.sh_base], a[u] * mag);
            else atomic_add_noret(&S.ub[j[u]], a[u] * mag);
        }
    }
}
// |zhat'_new - zhat'_old|, rounded up
__device__ __forceinline__ double change_mag(double znew, double zold) {
    return fabs(znew - zold) * (1.0 + 0x1p-40);
}

// Row sums of a light tile.  FP64 sweeps gather zhat'; fixed-point sweeps
// gather the 32-bit copy, except for rows the copy cannot resolve
// (fix_too_coarse), which gather zhat' (flags in LDS, checked per arc only
// when the tile holds such a row).  rd: the lane's row data (lane < nrows).
template <bool MIRROR>
__device__ __forceinline__ double light_tile_sums(const int32_t* __restrict__ prow_ptr, const int32_t* __restrict__ pcol,
                                                  const float* __restrict__ pw, const SorState& S, int32_t r0,
                                                  int nrows, const RowData& rd, int* pre, double* acc, int* flag,
                                                  const int* must = nullptr) {
    const double* __restrict__ zh = S.zh;
    const int32_t* __restrict__ zq = S.zq;
    const int lane = lane_id();
    auto arc64 = [&](int k) {
        double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
        return a * zh[__builtin_nontemporal_load(&pcol[k])];
    };
    if (must) {  // only the rows that must be swept gather (wave-uniform branch)
        if constexpr (MIRROR) {
            flag[lane] = lane < nrows && fix_too_coarse(rd, S.epsp) ? 1 : 0;
            auto arcq = [&](int k) {
                double a = pw ? static_cast<double>(__builtin_nontemporal_load(&pw[k])) : 1.0;
                return a * fix_dec(zq[__builtin_nontemporal_load(&pcol[k])]);
            };
            return tile_row_sums(prow_ptr, r0, nrows, pre, acc, [&](int k, int slot) {
                return must[slot] ? (flag[slot] ? arc64(k) : arcq(k)) : 0.0;
            });
        } else {
            return tile_row_sums(prow_ptr, r0, nrows, pre, acc,
                                 [&](int k, int slot) { return must[slot] ? arc64(k) : 0.0; });
        }
    }
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
    const int wid = wave_id(), lane = lane_id();
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

// One light tile (rows tv.tile_start[tix] .. tv.tile_start[tix + 1] - 1) of
// k_sor_class, taken by the whole wave; md is the sweep's mode.  pre, acc,
// flag and mustb are the wave's LDS scratch.
template <bool MIRROR, bool SHADOW, bool SKIP>
__device__ __forceinline__ void sor_light_tile(int64_t tix, int md, const TileView& tv,
                                               const int32_t* __restrict__ prow_ptr, const int32_t* __restrict__ pcol,
                                               const float* __restrict__ pw, const SorState& S, int* updated, int* bad,
                                               unsigned long long* stats, int* pre, double* acc, int* flag,
                                               int* mustb) {
    const int lane = lane_id();
    if (tv.tile_heavy[tix] >= 0) return;  // taken by the chunk waves
    const int32_t r0 = tv.tile_start[tix];
    const int nrows = tv.tile_start[tix + 1] - r0;
    RowData rd{};
    if (lane < nrows) rd = row_load(r0 + lane, S);
    const int* must = nullptr;
    bool sweep_row = lane < nrows;
    if (SKIP && md == 2) {
        const int64_t i = r0 + lane;
        sweep_row = lane < nrows && !bound_quiet(S.ub[i], rd, S);
        const uint64_t skipped = __ballot(lane < nrows && !sweep_row);
        if (skipped) {  // skipped rows and their arcs (counters 2 and 3 or 4)
            int d = lane < nrows && !sweep_row ? prow_ptr[i + 1] - prow_ptr[i] : 0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
            if (lane == 0) {
                stripe_add(stats, 2, static_cast<unsigned long long>(__popcll(skipped)));
                stripe_add(stats, MIRROR ? 3 : 4, static_cast<unsigned long long>(d));
            }
        }
        if (!__ballot(sweep_row)) {  // the whole tile is quiet
            if (lane < nrows) keep_row<SHADOW>(r0 + lane, rd, S);
            return;
        }
        mustb[lane] = sweep_row ? 1 : 0;
        wave_sync_lds();
        must = mustb;
    }
    const double sum = light_tile_sums<MIRROR>(prow_ptr, pcol, pw, S, r0, nrows, rd, pre, acc,
                                               flag, must);
    bool upd = false, nonfinite = false;
    double rr = 0.0, zn = 0.0;
    if (sweep_row) upd = sor_row_with<SHADOW>(r0 + lane, rd, sum, S, &nonfinite, &rr, &zn);
    else if (lane < nrows) keep_row<SHADOW>(r0 + lane, rd, S);
    uint64_t um = __ballot(upd);
    if (__ballot(nonfinite) && lane == 0) flag_set(bad);
    if (um && lane == 0) {
        flag_set(updated);
        stripe_add(stats, 0, static_cast<unsigned long long>(__popcll(um)));
    }
    if (SKIP && md >= 1) {
        // the swept rows' own bounds; then the neighbours of the updated rows,
        // the whole wave taking one row at a time
        if (sweep_row) S.ub[r0 + lane] = own_bound(rr, upd, S.omega, rd.opd);
        const double mag = upd ? change_mag(zn, rd.z) : 0.0;
        // each updated row's range in the bound CSR, loaded by its own lane
        // at once rather than row by row inside the loop
        int bb = 0, be = 0;
        if (upd) {
            bb = S.brow[r0 + lane];
            be = S.brow[r0 + lane + 1];
        }
        unsigned long long adds = 0;
        for (uint64_t rem = um; rem; rem &= rem - 1) {
            const int l = __builtin_ctzll(rem);
            const int b = __shfl(bb, l, 64), e = __shfl(be, l, 64);
            bound_arcs<4, SHADOW>(S, b, e, __shfl(mag, l, 64));
            adds += static_cast<unsigned long long>(e - b);
        }
        if (adds && lane == 0) stripe_add(stats, 5, adds);  // counter 5: bound additions
    }
}

// Bound skipping with GT consecutive tiles per wave: one lane per row over
// the group's rows (consecutive, at most 64 GT), so a quiet group costs one
// round of coalesced loads instead of GT waves.  Returns the mask of tiles
// holding a light row that is not provably quiet; sor_light_tile then sweeps
// those tiles, repeating the check for its own rows.  The light rows of the
// other tiles are counted as skipped here (and written to the shadow arrays
// in a merged tail).  Heavy rows belong to their chunk waves.
template <bool MIRROR, bool SHADOW, int GT>
__device__ __forceinline__ uint32_t light_group_check(const TileView& tv, int64_t ta, int nt,
                                                      const int32_t* __restrict__ prow_ptr, const SorState& S,
                                                      unsigned long long* stats) {
    constexpr int kSlices = GT;  // a tile holds at most 64 rows
    const int lane = lane_id();
    // lane q <= nt: first row of tile ta + q (lane nt: one past the group)
    const int32_t ts = lane <= nt ? tv.tile_start[ta + lane] : 0;
    int32_t tsk[GT + 1];  // the same, in every lane (all lanes are active here)
#pragma unroll
    for (int k = 0; k <= GT; ++k) tsk[k] = __shfl(ts, k, 64);
    const int32_t R0 = tsk[0], R1 = __shfl(ts, nt, 64);
    int tq[kSlices];     // the lane's row's tile within the group, -1: none or heavy
    int dg[kSlices];     // its arc count
    double zk[kSlices];  // its value (shadow copy of a merged tail)
    uint32_t active = 0u;
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
        tq[sl] = -1;
        dg[sl] = 0;
        zk[sl] = 0.0;
        const int32_t i = R0 + 64 * sl + lane;
        if (R0 + 64 * sl >= R1) continue;  // uniform
        bool nq = false;
        if (i < R1) {
            const int d = prow_ptr[i + 1] - prow_ptr[i];
            if (d <= kArcBudget) {
                const double sp = __builtin_nontemporal_load(&S.sp[i]);
                const double opd = __builtin_nontemporal_load(&S.popd[i]);
                if constexpr (SHADOW) zk[sl] = __builtin_nontemporal_load(&S.zh[i]);
                nq = !(S.ub[i] + resid_err(opd) < 0.999 * S.thr * S.epsp * sp);
                int q = 0;
#pragma unroll
                for (int k = 1; k < GT; ++k) q += k < nt && i >= tsk[k] ? 1 : 0;
                tq[sl] = q;
                dg[sl] = d;
            }
        }
        if (__ballot(nq))
            for (int q = 0; q < nt; ++q)
                if (__ballot(nq && tq[sl] == q)) active |= 1u << q;
    }
    // the light rows of the tiles left out: skipped
    unsigned long long rows = 0, arcs = 0;
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
        const bool skip = tq[sl] >= 0 && !((active >> tq[sl]) & 1u);
        if (skip) {
            ++rows;
            arcs += static_cast<unsigned long long>(dg[sl]);
            if constexpr (SHADOW) {
                const int64_t i = R0 + 64 * sl + lane;
                S.zsh[i - S.sh_base] = zk[sl];
                S.zqsh[i - S.sh_base] = fix_enc(zk[sl]);
            }
        }
    }
    if (__ballot(rows != 0)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            rows += __shfl_xor(rows, o, 64);
            arcs += __shfl_xor(arcs, o, 64);
        }
        if (lane == 0) {
            stripe_add(stats, 2, rows);
            stripe_add(stats, MIRROR ? 3 : 4, arcs);
        }
    }
    return active;
}

// One colour class in a single launch: the first nchunks waves each sum one
// heavy-row chunk (combined as above), the rest take one light tile each.
// Used when no heavy row of the class has more than kMaxPackedChunks chunks.
// SHADOW: the launch covers several trailing classes at once (a merged tail);
// rows write to the shadow arrays and k_sor_commit publishes them afterwards,
// so within the launch every gather sees values from before it.
// A sweep that follows a quiet sweep (no row updated) would change nothing:
// when *prev is 0 the launch returns at once.
// SKIP: the variant with bound skipping, whose sweep mode is *mode.
// GT > 1 (with SKIP): each light wave takes GT consecutive tiles.
constexpr int kSkipGroupTiles = 8;
template <bool MIRROR, bool SHADOW, bool SKIP, int GT = 1>
__global__ __launch_bounds__(kBlock) void k_sor_class(TileView tv, const int32_t* __restrict__ prow_ptr,
                                                      const int32_t* __restrict__ pcol, const float* __restrict__ pw,
                                                      SorState S, const int* prev, int* updated, int* bad,
                                                      unsigned long long* stats, const int* __restrict__ mode) {
    __shared__ int s_pre[kWavesPerBlock][65];
    __shared__ double s_acc[kWavesPerBlock][64];
    __shared__ int s_flag[kWavesPerBlock][64];
    __shared__ int s_must[kWavesPerBlock][64];
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    // 0 plain, 1 bounds, 2 bounds and skipping (bound skipping); read before any
    // other load so that the branches on it wait for nothing else
    int md = 0;
    if constexpr (SKIP) md = *mode;
    const int wid = wave_id(), lane = lane_id();
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
        // a heavy row whose bound shows it quiet is skipped by all its chunk
        // waves alike (nothing writes its bound during the launch before its
        // chunks have all arrived, and a skipped row has no arrivals)
        RowData rd{};
        if (SKIP && md == 2) {
            rd = row_load(row, S);  // the same address in every lane
            if (bound_quiet(S.ub[row], rd, S)) {
                if (lane == 0 && cidx == tv.heavy_chunk0[h]) {
                    stripe_add(stats, 2, 1ull);  // heavy rows' skipped arcs: counter 6 or 4
                    stripe_add(stats, MIRROR ? 6 : 4,
                               static_cast<unsigned long long>(prow_ptr[row + 1] - prow_ptr[row]));
                    if constexpr (SHADOW) keep_row<SHADOW>(row, rd, S);
                }
                return;
            }
        } else if (lane == 0) {
            rd = row_load(row, S);
        }
        const double part = chunk_sum(beg, end, arc64);
        int fin_upd = 0;
        double mag = 0.0;
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
                double rr = 0.0, zn = 0.0;
                bool upd = sor_row_with<SHADOW>(row, rd, tot, S, &nonfinite, &rr, &zn);
                if (nonfinite) flag_set(bad);
                if (upd) {
                    flag_set(updated);
                    stripe_add(stats, 0, 1ull);
                    fin_upd = 1;
                }
                if (SKIP && md >= 1) {  // the row's own bound
                    S.ub[row] = own_bound(rr, upd, S.omega, rd.opd);
                    if (upd) mag = change_mag(zn, rd.z);
                }
            }
        }
        // an updated heavy row raises its neighbours' bounds, the whole wave taking its arcs
        if (SKIP && md >= 1 && __shfl(fin_upd, 0, 64)) {
            bound_arcs<16, SHADOW>(S, S.brow[row], S.brow[row + 1], __shfl(mag, 0, 64));
            if (lane == 0) stripe_add(stats, 5, static_cast<unsigned long long>(S.brow[row + 1] - S.brow[row]));
        }
        return;
    }
    wv -= tv.nchunks;
    if constexpr (GT == 1) {
        if (wv >= tv.ntiles) return;
        sor_light_tile<MIRROR, SHADOW, SKIP>(tv.t0 + wv, md, tv, prow_ptr, pcol, pw, S, updated, bad, stats,
                                             s_pre[wid], s_acc[wid], s_flag[wid], s_must[wid]);
    } else {
        // GT consecutive tiles per wave: the launch shape for sweeps expected
        // to skip; in modes 0 and 1 the wave sweeps its tiles one by one
        const int64_t ta = tv.t0 + wv * GT;
        const int64_t tend = tv.t0 + tv.ntiles;
        if (ta >= tend) return;
        const int nt = static_cast<int>(min(static_cast<int64_t>(GT), tend - ta));
        uint32_t active = nt >= 32 ? ~0u : (1u << nt) - 1u;
        if (md == 2) active = light_group_check<MIRROR, SHADOW, GT>(tv, ta, nt, prow_ptr, S, stats);
        for (; active; active &= active - 1u)
            sor_light_tile<MIRROR, SHADOW, SKIP>(ta + __builtin_ctz(active), md, tv, prow_ptr, pcol, pw, S, updated,
                                                 bad, stats, s_pre[wid], s_acc[wid], s_flag[wid], s_must[wid]);
    }
}

// Start of sweep `sw` with bound skipping.  The mode: 0 while `allow` is 0
// (first sweep of a phase) or the previous sweep updated `limit` rows or
// more; otherwise 1 (bounds only: every row is swept, so every bound is set
// afterwards) after a sweep in mode 0, else 2 (bounds and skipping).  The
// update count comes from the striped counters, remembered per sweep in
// snaps.  Entering mode 1 clears the merged tail's collected adds; mode 2
// first adds those of the previous sweep's merged-tail launch to the tail
// rows' bounds.  Every block takes the same decision; block 0 records it.
// Returns at once after a quiet sweep.
__global__ void k_sweep_begin(const int* prev, int64_t sw, double* ub, double* ub_tail, int64_t tail_start,
                              int64_t n, const unsigned long long* stats, unsigned long long* snaps, int* modes,
                              int allow, double limit) {
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    __shared__ int s_mode[2];
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < kStripes; ++k) tot += stats[k * kStripeStride];
        int m = 0, pm = 0;
        if (allow) {
            pm = modes[sw - 1];
            if (static_cast<double>(tot - snaps[sw - 1]) < limit) m = pm >= 1 ? 2 : 1;
        }
        s_mode[0] = m;
        s_mode[1] = pm;
        if (blockIdx.x == 0) {
            snaps[sw] = tot;
            modes[sw] = m;
        }
    }
    __syncthreads();
    const int m = s_mode[0], pm = s_mode[1];
    if (m == 0) return;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n - tail_start;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (pm != 0) ub[tail_start + t] += ub_tail[t];
        ub_tail[t] = 0.0;
    }
}

// Start of a sweep of the plain kernel while bound skipping is enabled:
// records the update count so far and mode 0, so that the sweep after it
// may start the bounds.
__global__ void k_sweep_snap(const int* prev, int64_t sw, const unsigned long long* stats, unsigned long long* snaps,
                             int* modes) {
    if (prev && __atomic_load_n(prev, __ATOMIC_RELAXED) == 0) return;
    if (threadIdx.x != 0) return;
    unsigned long long tot = 0;
    for (int k = 0; k < kStripes; ++k) tot += stats[k * kStripeStride];
    snaps[sw] = tot;
    modes[sw] = 0;
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
    const int wid = wave_id(), lane = lane_id();
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
