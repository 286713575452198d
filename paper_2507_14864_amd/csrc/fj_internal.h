// Internal declarations shared by the libfj translation units (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fj.h"

namespace fj {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block for the tile kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kStripes = 64;       // striped global counters (one 128 B line each)
constexpr int kStripeStride = 16;  // u64 per stripe line
constexpr int kMaxColours = 2048;  // colour classes supported by the permutation pass
// bound skipping starts once a sweep updated fewer than this fraction of the rows
constexpr double kSkipBelow = 0.05;
// by default only on graphs with at least this many stored arcs: below it a
// sweep is bound by its launches, and the per-sweep bookkeeping launch and the
// heavier kernel variant cost more than the skipped gathers save
constexpr int64_t kSkipMinArcs = int64_t{1} << 24;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
fj_status hip_fail(hipError_t e, const char* what);
#define FJ_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::fj::hip_fail(e_, #call);        \
    } while (0)

// ------------------------------------------------------ workspace carving
struct Carver {
    char* base;       // nullptr for a size query
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Work partition of a CSR row range for wave-level kernels.
//  - Light tiles: at most 64 consecutive rows and fewer than 2*kArcBudget arcs
//    (a tile starts at every 64th row, wherever floor(row_ptr/kArcBudget)
//    changes, at every segment start, and around every heavy row).
//  - Heavy rows: more than kArcBudget arcs.  Each is a tile of its own and is
//    split into chunks of kArcBudget arcs; partial sums per chunk are combined
//    in chunk order by a second launch.
// Segments (colour classes, or one segment for the whole graph) never share a
// tile; per-segment offsets into every list are kept on the host.
constexpr int kArcBudget = 256;
// rows longer than this are reduced by a whole block in the persistent sweep
constexpr int kBigRow = 2048;
// heavy-row chunks combined inside one sweep launch: the low kPackedCountBits
// of a row's 64-bit accumulator count arrivals, so a row may have at most
// kMaxPackedChunks chunks for its colour class to be swept in one launch
constexpr int kPackedCountBits = 12;
constexpr int kMaxPackedChunks = (1 << kPackedCountBits) - 1;
// colour classes holding less than this fraction of the arcs may be swept together
constexpr double kMergeArcFraction = 0.01;

struct TileSet {
    int64_t ntiles = 0, nheavy = 0, nchunks = 0;
    int32_t* tile_start = nullptr;   // [ntiles + 1]
    int32_t* tile_heavy = nullptr;   // [ntiles] heavy index of a heavy tile, else -1
    int32_t* heavy_row = nullptr;    // [nheavy]
    int32_t* heavy_chunk0 = nullptr; // [nheavy + 1]
    int32_t* chunk_heavy = nullptr;  // [nchunks] heavy index owning the chunk
    int32_t* chunk_beg = nullptr;    // [nchunks] first arc of the chunk
    int32_t* chunk_end = nullptr;    // [nchunks] one past the last arc of the chunk
    std::vector<int64_t> seg_tile, seg_heavy, seg_chunk;  // [nseg + 1] host offsets
    int64_t* d_seg_tile = nullptr;   // device copies of seg_tile / seg_heavy
    int64_t* d_seg_heavy = nullptr;
};

// Kernel-argument view of one segment of a TileSet (or of all of it).
struct TileView {
    const int32_t* tile_start;
    const int32_t* tile_heavy;
    const int32_t* heavy_row;
    const int32_t* heavy_chunk0;
    const int32_t* chunk_heavy;
    const int32_t* chunk_beg;
    int64_t t0, ntiles;  // tiles [t0, t0 + ntiles)
    int64_t c0, nchunks; // heavy chunks [c0, c0 + nchunks)
    int64_t h0, h1;      // heavy rows [h0, h1)
    const int32_t* chunk_end;
};

inline TileView tile_view(const TileSet& T, int seg) {
    TileView v{T.tile_start, T.tile_heavy, T.heavy_row, T.heavy_chunk0, T.chunk_heavy, T.chunk_beg,
               T.seg_tile[seg], T.seg_tile[seg + 1] - T.seg_tile[seg],
               T.seg_chunk[seg], T.seg_chunk[seg + 1] - T.seg_chunk[seg],
               T.seg_heavy[seg], T.seg_heavy[seg + 1], T.chunk_end};
    return v;
}
inline TileView tile_view_all(const TileSet& T) {
    TileView v{T.tile_start, T.tile_heavy, T.heavy_row, T.heavy_chunk0, T.chunk_heavy, T.chunk_beg,
               0, T.ntiles, 0, T.nchunks, 0, T.nheavy, T.chunk_end};
    return v;
}
inline unsigned waves_to_blocks(int64_t waves) {
    return static_cast<unsigned>((waves + kWavesPerBlock - 1) / kWavesPerBlock);
}

}  // namespace fj

// Host object behind fj_graph*.
struct fj_graph {
    int64_t n = 0, nnz = 0;
    int directed = 0, weighted = 0;
    int32_t max_degree = 0, max_in_degree = 0;
    // CSR(A), caller-owned
    const int32_t* row_ptr = nullptr;
    const int32_t* col = nullptr;
    const float* w = nullptr;
    // CSR(A^T): aliases CSR(A) when undirected
    const int32_t* t_row_ptr = nullptr;
    const int32_t* t_col = nullptr;
    const float* t_w = nullptr;
    // per node, original labels
    double* opd = nullptr;   // 1 + d_i
    double* inv64 = nullptr; // 1 / (1 + d_i)
    float* inv32 = nullptr;
    // colour-ordered copy (FJ_GRAPH_COLOUR)
    int32_t num_colours = 0, colour_rounds = 0;
    std::vector<int64_t> class_off;  // [num_colours + 1] host copy
    std::vector<uint8_t> class_packed;  // [num_colours] 1: no heavy row has more than kMaxPackedChunks chunks
    // Tail merge (undirected graphs): classes [merge_min, num_colours) are each
    // under kMergeArcFraction of the arcs; merge_coupling[T] (T >= merge_min) is
    // max over rows i in classes >= T of sum_{j in classes >= T} a_ij / (1 + d_i).
    int32_t merge_min = 0;
    std::vector<double> merge_coupling;
    // every heavy row of CSR(A) has at most kMaxPackedChunks chunks (gather-form rounds possible)
    int a_packed = 0;
    int32_t* colour = nullptr;       // [n] original labels
    int32_t* perm = nullptr;         // new -> old
    int32_t* iperm = nullptr;        // old -> new
    int32_t* prow_ptr = nullptr;     // relabelled CSR(A)
    int32_t* pcol = nullptr;
    float* pw = nullptr;
    int32_t* qrow_ptr = nullptr;     // relabelled CSR(A^T), directed graphs: row i lists
    int32_t* qcol = nullptr;         // the rows of A that read zhat'_i, with a_ji
    float* qw = nullptr;
    double* popd = nullptr;          // 1 + d, relabelled
    double* pinv64 = nullptr;
    // wave work partitions
    fj::TileSet tiles_a;   // CSR(A), original labels (certificate, measures)
    fj::TileSet tiles_t;   // CSR(A^T), original labels (push); same as tiles_a when undirected
    fj::TileSet tiles_p;   // relabelled CSR(A), one segment per colour class (SOR)
    int64_t heavy_arcs_p = 0;  // arcs of the rows tiles_p splits into chunks (always gathered in FP64)
};

namespace fj {

// Kernel launchers (fj_graph.hip).  Besides the public flags, graph_build
// takes kGraphNoBoundCsr: a directed coloured graph then skips the relabelled
// CSR(A^T) that only the single-graph sweeps' bound skipping reads.
constexpr int32_t kGraphNoBoundCsr = 1 << 16;
fj_status graph_build(fj_graph* g, const fj_graph_desc* d, int32_t flags, void* ws, size_t ws_bytes,
                      hipStream_t st);
size_t graph_ws_bytes(const fj_graph_desc* d, int32_t flags);

// Measures for fj_solve_opts.measures (fj_metrics.hip), in a workspace of
// measures_ws_bytes: all passes over z, or the node passes with D's per-block
// sums over every stored arc already in part_d[nbd].
size_t measures_ws_bytes(const fj_graph* g);
fj_status measures_full(const fj_graph* g, const double* s, const double* z, void* ws, hipStream_t st,
                        fj_metrics_out* out);
fj_status measures_with_d(const fj_graph* g, const double* s, const double* z, const double* part_d, int64_t nbd,
                          void* ws, hipStream_t st, fj_metrics_out* out);

// Scan helper (fj_graph.hip): exclusive scan of int32 in -> out (may alias), n entries,
// returns total through *total_dev (device int64) when not null. tmp: scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
size_t certify_ws_bytes(const fj_graph* g);
// max_v |s_v - ((I+L) z)_v| / (s_v + c) in FP64 (certificate kernels); synchronizes st
fj_status residual_level(const fj_graph* g, const double* s, const double* z, double c, void* ws, size_t ws_bytes,
                         hipStream_t st, double* tau);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* tmp, hipStream_t st);

}  // namespace fj
