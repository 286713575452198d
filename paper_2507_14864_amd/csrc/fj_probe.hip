// Diagnostic: the random-gather ceiling of the sweep's memory access pattern.
//
// A colour-class sweep (Eq. (sor1) in pull form) streams the column indices of
// its rows and gathers one value of the estimate per arc; almost all of its
// time goes to those gathers, whose targets are spread over the whole node
// range.  This kernel performs exactly that access stream and nothing else:
// every arc of the colour-major CSR loads its column index with a streaming
// load and gathers the value at that index (4-byte fixed-point copy or 8-byte
// FP64 estimate), with four loads in flight per lane as in the sweep, and no
// per-row reduction or update.  Its rate is what a sweep can reach at best on
// this graph; the ratio of the sweep's arc rate to it shows how much of the
// sweep's time is spent outside the gathers.
#include <algorithm>

#include "fj_device.h"
#include "fj_internal.h"

namespace fj {
namespace {

constexpr int kProbeUnroll = 4;

template <typename V>
__global__ __launch_bounds__(kBlock) void k_gather_probe(int64_t nnz, const int32_t* __restrict__ col,
                                                         const V* __restrict__ vals, unsigned long long* sink) {
    const int lane = lane_id();
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * kBlock) >> 6;
    constexpr int64_t kStep = 64 * kProbeUnroll;
    unsigned long long acc = 0;
    for (int64_t base = wave * kStep; base < nnz; base += nwaves * kStep) {
        V v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const int64_t k = base + 64 * u + lane;
            v[u] = k < nnz ? vals[__builtin_nontemporal_load(&col[k])] : V(0);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            unsigned long long bits = 0;
            __builtin_memcpy(&bits, &v[u], sizeof(V));
            acc += bits;
        }
    }
    // one store per wave keeps the loads live
    acc = static_cast<unsigned long long>(wave_sum_ll(static_cast<long long>(acc)));
    if (lane == 0) sink[wave] = acc;
}

struct ProbeLayout {
    void* vals;
    unsigned long long* sink;
};

constexpr int kProbeWavesPerCU = 32;
constexpr int kProbeCUs = 256;

int64_t probe_waves(int64_t nnz) {
    const int64_t need = (nnz + 64 * kProbeUnroll - 1) / (64 * kProbeUnroll);
    return std::max<int64_t>(1, std::min<int64_t>(need, static_cast<int64_t>(kProbeCUs) * kProbeWavesPerCU));
}

ProbeLayout carve_probe(Carver& cv, const fj_graph* g) {
    ProbeLayout L{};
    L.vals = cv.take<double>(g->n + 1);
    L.sink = cv.take<unsigned long long>(probe_waves(g->nnz) + kWavesPerBlock);
    return L;
}

}  // namespace
}  // namespace fj

using namespace fj;

extern "C" size_t fj_gather_probe_workspace_bytes(const fj_graph* g) {
    if (!g) return 0;
    Carver cv(nullptr);
    carve_probe(cv, g);
    return cv.bytes();
}

extern "C" fj_status fj_gather_probe(const fj_graph* g, int32_t value_bytes, int32_t reps, double* arcs_per_s,
                                     void* ws, size_t ws_bytes, void* stream) {
    if (!g || !arcs_per_s || !ws || (value_bytes != 4 && value_bytes != 8) || reps < 1 || reps > 1000) {
        set_error("fj_gather_probe: bad argument (value_bytes 4 or 8, reps 1..1000)");
        return FJ_ERR_INVALID_ARGUMENT;
    }
    if (ws_bytes < fj_gather_probe_workspace_bytes(g)) {
        set_error("fj_gather_probe: workspace too small");
        return FJ_ERR_WORKSPACE_TOO_SMALL;
    }
    *arcs_per_s = 0.0;
    if (g->nnz == 0) return FJ_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    const ProbeLayout L = carve_probe(cv, g);
    // the colour-major copy when there is one (the order the sweeps read)
    const int32_t* col = g->num_colours > 0 ? g->pcol : g->col;
    FJ_HIP(hipMemsetAsync(L.vals, 0, sizeof(double) * (g->n + 1), st));
    const unsigned blocks = waves_to_blocks(probe_waves(g->nnz));
    auto launch = [&]() {
        if (value_bytes == 4)
            hipLaunchKernelGGL(k_gather_probe<int32_t>, dim3(blocks), dim3(kBlock), 0, st, g->nnz, col,
                               static_cast<const int32_t*>(L.vals), L.sink);
        else
            hipLaunchKernelGGL(k_gather_probe<double>, dim3(blocks), dim3(kBlock), 0, st, g->nnz, col,
                               static_cast<const double*>(L.vals), L.sink);
    };
    launch();  // warm-up: the index stream and the values reach their steady cache state
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    fj_status rc = FJ_OK;
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = hip_fail(e, "fj_gather_probe");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != FJ_OK) return rc;
    *arcs_per_s = ms > 0.f ? static_cast<double>(g->nnz) * reps / (static_cast<double>(ms) * 1e-3) : 0.0;
    return FJ_OK;
}
