/*
 * fj.h -- C ABI of libfj.so: the Friedkin-Johnsen equilibrium z = (I+L)^{-1} s
 * by residual push with over-relaxation on MI355X (gfx950), and the Table 1
 * measures over z.
 *
 * Method: "Efficient Algorithms for Relevant Quantities of Friedkin-Johnsen
 * Opinion Dynamics Model" (arXiv 2507.14864): Lemma 1 (definition of z),
 * Alg. 1-3 (BoundLocalIter, ImprovedBLI, BoundLocalIterSOR), Lemma 4
 * (residual invariant), Lemma 7 (relative-error certificate), Thm. 8 (push
 * equals Gauss-Seidel), Eqs. (sor1)-(sor3), Table 1 (measures).
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *    tensor's data_ptr) unless the comment says [host].
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *  - The library never allocates device memory at run time (its only device
 *    memory of its own is the static 8 MiB array of fj_metrics_noalloc, part
 *    of its code object).  Callers query the workspace size of each call and
 *    pass a buffer of at least that many bytes, aligned to 256 bytes.  A graph workspace must stay alive and untouched while the
 *    graph handle exists.  A solve/metrics workspace may be reused between
 *    calls but not by two concurrent calls.
 *  - Graph: CSR of the adjacency matrix A.  Row i lists the nodes j with
 *    a_ij > 0, i.e. the nodes node i listens to (the sum of Eq. (1)).
 *    d_i = sum_j a_ij and L = D - A (Sec. 3.2).  Rows must be strictly
 *    increasing in column, without self-loops; weights (optional) finite and
 *    > 0.  An undirected graph stores every edge in both rows with equal
 *    weights.  Indices are int32, so nnz < 2^31.
 *  - Every call returns an fj_status; no exception crosses the ABI.  On an
 *    error other than FJ_ERR_NOT_CONVERGED, outputs are left untouched;
 *    fj_last_error() returns a message for the calling thread.
 */
#ifndef FJ_H
#define FJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fj_status;
#define FJ_OK 0
#define FJ_ERR_INVALID_ARGUMENT 1
#define FJ_ERR_WORKSPACE_TOO_SMALL 2
#define FJ_ERR_NOT_CONVERGED 3
#define FJ_ERR_HIP 4
#define FJ_ERR_UNSUPPORTED 5

/* Thread-local message for the last non-OK status returned on this thread. */
const char* fj_last_error(void);

/* Library version, for the Python binding's sanity check. */
int32_t fj_version(void);

/* ------------------------------------------------------------------ graph */

typedef struct fj_graph fj_graph; /* opaque host object referencing device buffers */

typedef struct {
    int64_t n;              /* nodes */
    int64_t nnz;            /* stored arcs = row_ptr[n] */
    const int32_t* row_ptr; /* device [n+1], row_ptr[0] = 0, nondecreasing */
    const int32_t* col;     /* device [nnz] */
    const float* w;         /* device [nnz] weights a_ij, or NULL for unit weights */
    int32_t directed;       /* 0: A must be symmetric (checked by fj_graph_create) */
} fj_graph_desc;

/* fj_graph_create flags */
#define FJ_GRAPH_COLOUR 1 /* also build the colour-ordered copy used by FJ_SCHED_SOR */

/* Bytes of graph workspace fj_graph_create needs for this desc and flags. */
size_t fj_graph_workspace_bytes(const fj_graph_desc* desc, int32_t flags);

/* Validate the CSR (indices in range, rows strictly increasing, no self-loops,
 * positive finite weights, symmetry when undirected), then build what the
 * solver needs in `ws`: d and 1/(1+d) (Sec. 3.2); for directed graphs the CSR
 * of A^T (a push at v feeds every u with a_uv > 0, the column of A in the
 * proof of Lemma 4); with FJ_GRAPH_COLOUR a colouring of the symmetrised
 * pattern A + A^T and a relabelled copy of A whose colour classes are
 * contiguous (the order the SOR sweeps visit, Thm. 8 with Eq. (sor1)), on a
 * directed graph with a relabelled copy of A^T beside it (the rows whose
 * residual bounds an update raises, fj_solve_opts.skip_below); on an
 * undirected graph also, for the trailing small classes, the coupling bound
 * that decides whether a solve may sweep them together (fj_solve_opts).
 * The caller's row_ptr/col/w must outlive the handle.  Synchronizes `stream`.
 * Errors: FJ_ERR_INVALID_ARGUMENT (bad desc or CSR), FJ_ERR_WORKSPACE_TOO_SMALL,
 * FJ_ERR_UNSUPPORTED (more colours than supported), FJ_ERR_HIP. */
fj_status fj_graph_create(const fj_graph_desc* desc, int32_t flags, void* ws, size_t ws_bytes,
                          void* stream, fj_graph** out);

/* Free the host object (the caller frees the workspace). NULL is accepted. */
fj_status fj_graph_destroy(fj_graph* g);

typedef struct {
    int64_t n, nnz;
    int32_t directed, weighted;
    int32_t max_degree;    /* longest row of A */
    int32_t max_in_degree; /* longest row of A^T */
    int32_t num_colours;   /* 0 when built without FJ_GRAPH_COLOUR */
    int32_t colour_rounds; /* priority levels of the parallel colouring (one launch each) */
} fj_graph_info;

/* [host] out. */
fj_status fj_graph_get_info(const fj_graph* g, fj_graph_info* out);

/* Colour classes: sizes[k] for k < num_colours, [host] out with room for
 * num_colours entries.  FJ_ERR_INVALID_ARGUMENT if the graph has no colouring. */
fj_status fj_graph_colour_sizes(const fj_graph* g, int64_t* sizes);

/* Device copy of the colour of every node (original labels), int32 [n]. */
fj_status fj_graph_colours(const fj_graph* g, int32_t* colours, void* stream);

/* ------------------------------------------------------------------ solve */

#define FJ_FP32 0 /* FP32 residual pushes; FP64 estimate, certificate and measures */
#define FJ_FP64 1 /* FP64 throughout */

#define FJ_SCHED_AUTO 0 /* SOR when the graph has a colouring, else PUSH */
#define FJ_SCHED_PUSH 1 /* frontier push rounds (Alg. 1 order relaxed to rounds), omega in (0,1] */
#define FJ_SCHED_SOR 2  /* colour-ordered over-relaxed sweeps, omega in (0,2); needs FJ_GRAPH_COLOUR */

/* Table 1 measures of an opinion vector (fj_metrics, fj_solve_opts.measures). */
typedef struct {
    double P;    /* polarization  sum_i (z_i - mean)^2                      (Table 1) */
    double D;    /* disagreement  sum over edges of a_ij (z_i - z_j)^2; an undirected
                    edge counts once, a directed arc once                  (Table 1) */
    double I;    /* internal conflict sum_i (z_i - s_i)^2                    (Table 1) */
    double C;    /* controversy   sum_i z_i^2                                (Table 1) */
    double mean; /* 1^T z / n, the centring of Sec. 3.4 */
} fj_metrics_out;

typedef struct {
    double eps;   /* relative error target eps in (0,1) (Alg. 2 input) */
    double omega; /* relaxation factor (Alg. 3 input); 1 = BoundLocalIter */
    double c;     /* opinion shift of Alg. 2, >= 0 (paper: 1e-5) */
    double sigma; /* threshold of Alg. 2, > 0 (paper: 1e-5); eps' = sigma eps / (c + sigma) */
    int32_t precision; /* FJ_FP32 or FJ_FP64 */
    int32_t schedule;  /* FJ_SCHED_* */
    int64_t max_edge_visits; /* work cap; 0 selects 4096 * (nnz + n) */
    int32_t max_refinements; /* FP64 re-seeding passes after a failed certificate; <0 selects 8 */
    int32_t check_every;     /* rounds/sweeps between host checks of progress; <=0 selects 8 */
    const double* z0;        /* device [n] warm start (any vector, Lemma 4), or NULL */
    int32_t profile;         /* nonzero: time every launch of the iteration kernel with HIP
                                events on `stream` (adds small gaps between launches) */
    int32_t persistent;      /* nonzero: SOR runs as one cooperative launch with a grid
                                barrier per colour class instead of one launch per class */
    int32_t gather_bits;     /* FJ_FP32 sweeps: 0 or 32 = light rows gather the 32-bit fixed-point
                                copy of zhat' until quiet, then FP64; 64 = FP64 from the start.
                                The copy holds |zhat'| < 2: it is used only when s' = s + c and
                                the start are below 1.5, otherwise every sweep gathers FP64 */
    int32_t push_scatter;    /* FJ_SCHED_PUSH: 0 = rounds in gather form (each row recomputes its
                                residual from the round's start estimate), used when no row of A
                                exceeds 4095 x 256 arcs; 1 = every node above threshold scatters
                                omega r/(1+d) to its in-neighbours with atomics, found by a scan
                                of all nodes per round; 2 = rounds as in 1 while dense, then, once
                                a batch of check_every rounds averaged fewer than 2% of the nodes
                                pushing, over a frontier queue (Alg. 1's queue, as the round sets
                                of the proof of Thm. 5): a round pops only the nodes the previous
                                round lifted above threshold, appended by wave ballot and prefix
                                count, nodes bucketed by degree (a wave per 64 nodes, or a block
                                per node with more than 2048 arcs).  1 and 2 add in a
                                run-dependent order */
    int32_t no_tail_merge;   /* nonzero: one launch per colour class always.  Otherwise, on an
                                undirected graph, the trailing classes that each hold under 1% of
                                the arcs are swept by one launch (a Jacobi step among their rows)
                                when every such row's coupling to them, sum_j a_ij / (1 + d_i),
                                is below 0.9 (2/omega - 1): the Householder-John condition for
                                convergence of the resulting splitting */
    double skip_below;       /* FJ_SCHED_SOR, bound skipping.  From the
                                second batch of check_every sweeps on, a sweep that follows one
                                with fewer than skip_below * n updates keeps a bound on every row's residual: the
                                row's own |r| at its sweep ((1 - omega) |r| after its update,
                                Eq. (sor2)), raised by a_ij |change of zhat'_j| for each later
                                update of a node j that row i reads (Lemma 4; on a directed graph
                                the rows to raise come from the relabelled CSR(A^T)).  From the sweep after that, a
                                row whose bound, plus the rounding of its gathered sum, stays
                                below its update threshold keeps its value without gathering.
                                It would not have updated: the result is bit for bit the one
                                without skipping.  0 selects 0.05 on graphs of at least 2^24
                                stored arcs and no skipping on smaller ones (their sweeps are
                                bound by launches, which the bookkeeping only adds to);
                                positive: that fraction at any size; negative: never */
    fj_metrics_out* measures; /* [host] or NULL: also the Table 1 measures of the returned z, as
                                fj_metrics gives them (within rounding: the sums run in another
                                order).  FJ_SCHED_SOR forms D in the gather pass of its final
                                certificate, from the differences of zhat' (the shift cancels in
                                zhat'_i - zhat'_j), and only the node passes run after it; the
                                other schedules run fj_metrics' passes on z.  Written on FJ_OK
                                and FJ_ERR_NOT_CONVERGED.  fj_solve_batched ignores it */
} fj_solve_opts;

typedef struct {
    int64_t pushes;       /* node updates (pushes / row relaxations) */
    int64_t edge_visits;  /* arcs read by those updates (SOR: sweeps x nnz less the arcs of
                             skipped rows) */
    int64_t rounds;       /* push rounds or full sweeps */
    int64_t launches;     /* kernel launches of the iteration */
    int32_t refinements;  /* certificate failures that re-seeded the residual */
    int32_t certified;    /* 1 if max_v |r_v| / h_v <= 1 in FP64 at return */
    double max_ratio;     /* max_v |r_v| / h_v of the FP64 residual of the returned z */
    double seconds;       /* host wall time of the call */
    double kernel_ms;     /* profile mode: summed event time of the iteration kernel launches */
    int64_t kernel_launches; /* profile mode: launches timed */
    int32_t num_colours;  /* colour classes swept (SOR), 0 for push */
    int64_t mirror_rounds; /* SOR sweeps whose light rows gathered the 32-bit fixed-point copy;
                              push rounds with push_scatter = 2: rounds that popped a frontier queue */
    int32_t merged_classes; /* colour classes swept together as a merged tail (0: none) */
    int64_t skipped_rows;   /* row visits skipped by bound skipping */
    int64_t skipped_arcs;   /* the arcs of those rows */
    int64_t mirror_edge_visits; /* arcs gathered in the sweeps that read the fixed-point copy */
    int64_t bound_adds;     /* bound skipping: FP64 atomic additions to the residual bounds of the
                               rows that read an updated value (one per arc of an updated row) */
    int64_t mirror_fp64_edge_visits; /* of mirror_edge_visits, the arcs of rows with more than 256
                                        arcs, which gather the FP64 estimate in every sweep (rows
                                        the copy cannot resolve, also FP64, are not counted) */
} fj_solve_stats;

/* Bytes of solve workspace for this graph and options. */
size_t fj_solve_workspace_bytes(const fj_graph* g, const fj_solve_opts* opts);

/* ImprovedBLISOR (Alg. 2 around Alg. 3; Alg. 1 when omega = 1) on the GPU.
 * s: device [n] internal opinions, finite and >= 0 (Sec. 3.3; Lemma 6 needs
 * s >= 0); c = 0 needs min s > 0 (Sec. 5.1.3).  z: device [n] output.
 * On return with FJ_OK the FP64 residual r = s - (I+L) z satisfies
 * |r_v| <= eps' (s_v + c) for every v, which by Lemma 7 (with the shift of
 * Alg. 2) bounds |z - z_exact| <= eps' (z_exact + c) entrywise, hence relative
 * error <= eps wherever z_exact >= sigma.
 * FJ_ERR_NOT_CONVERGED: the work cap was hit, the iteration diverged (SOR with
 * omega > 1 on a directed graph is not guaranteed to converge), or the
 * refinement budget ran out; z then holds the last estimate and
 * stats->certified = 0.  stats: [host] or NULL.  Synchronizes `stream`.
 * Tracing: with FJ_TRACE set in the environment (to anything but empty or
 * 0), every host check of the iteration writes one JSON line to stderr --
 * {"fj_trace": "sor"|"push", "event": "batch", "mode", "rounds",
 * "batch_rounds", "updates", "edge_visits", "skipped_rows"} (cumulative counts)
 * -- and every FP64 certificate one {"event": "certificate", "rounds",
 * "max_ratio", "violations", "refinements"}. */
fj_status fj_solve(const fj_graph* g, const double* s, const fj_solve_opts* opts, double* z,
                   void* ws, size_t ws_bytes, fj_solve_stats* stats, void* stream);

/* ---------------------------------------------------- relaxation factor */

/* Eq. (optimal-omega): omega_opt = 1 + (mu / (1 + sqrt(1 - mu^2)))^2 for the
 * spectral radius mu = rho((I+D)^{-1} A) (Young's optimum for consistently
 * ordered matrices; a guide otherwise).  mu < 0 or NaN gives 1, mu >= 1 gives 2. */
double fj_optimal_omega(double mu);

size_t fj_omega_workspace_bytes(const fj_graph* g);

/* mu = rho((I+D)^{-1} A) by power iteration on the GPU (on the similar
 * symmetric matrix (I+D)^{-1/2} A (I+D)^{-1/2} when the graph is undirected),
 * from x0 = 1/sqrt(n), until two estimates 10 iterations apart differ by at
 * most tol * mu or max_iters (1..100000) iterations ran; then omega =
 * fj_optimal_omega(mu).  mu, omega, iters: [host] (iters may be NULL).
 * The estimate approaches mu from below when the second eigenvalue is close
 * to it.  Synchronizes `stream`. */
fj_status fj_estimate_omega(const fj_graph* g, int32_t max_iters, double tol, double* mu, double* omega,
                            int32_t* iters, void* ws, size_t ws_bytes, void* stream);

/* The paper's heuristic for omega (Sec. 5.2): solve with each candidate in
 * turn (fj_solve with opts, its omega replaced) and keep the candidate with
 * the fewest updates (stats.pushes); ties go to the smaller omega.
 * omegas: [host] n_omegas candidates.  updates, seconds: [host] n_omegas
 * outputs or NULL (updates -1 where the candidate did not certify).
 * z: device [n], holds the last candidate's result.  ws: a solve workspace
 * (fj_solve_workspace_bytes).  FJ_ERR_NOT_CONVERGED if no candidate certified. */
fj_status fj_tune_omega(const fj_graph* g, const double* s, const fj_solve_opts* opts, const double* omegas,
                        int32_t n_omegas, int64_t* updates, double* seconds, double* best_omega, double* z,
                        void* ws, size_t ws_bytes, void* stream);

/* --------------------------------------------------------------- measures */

size_t fj_metrics_workspace_bytes(const fj_graph* g);

/* FP64 reductions in a fixed order: bitwise reproducible for the same inputs.
 * s, z: device [n].  out: [host].  Synchronizes `stream`. */
fj_status fj_metrics(const fj_graph* g, const double* s, const double* z, fj_metrics_out* out,
                     void* ws, size_t ws_bytes, void* stream);

/* fj_metrics without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and the same fixed-order reductions as
 * fj_metrics (results bitwise equal), with their partial sums in a static
 * device array of fj_metrics_noalloc_max_bytes() = 8 MiB that the library
 * holds on every GPU it runs on until the process ends.  A graph needs
 * fj_metrics_noalloc_bytes(g) of it: 24 bytes per 4 wave tiles (a tile is at
 * most 64 rows or 256 arcs of a row) plus 72 bytes per 2048 nodes, about
 * 0.13 bytes per node plus 0.025 per arc (a 10M-node graph of 200M arcs
 * needs about 6 MB); a larger graph gets FJ_ERR_WORKSPACE_TOO_SMALL.  Calls nothing that allocates.  The array of the
 * current device is used, and `stream` (NULL: the null stream) must belong to
 * that device (else FJ_ERR_INVALID_ARGUMENT).  Every call on one GPU shares
 * its array: calls that overlap on one GPU (from several host threads or
 * streams) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero.  s, z: device [n]; out: [host].  Synchronizes
 * `stream`. */
size_t fj_metrics_noalloc_max_bytes(void);
size_t fj_metrics_noalloc_bytes(const fj_graph* g);
fj_status fj_metrics_noalloc(const fj_graph* g, const double* s, const double* z, fj_metrics_out* out,
                             void* stream);

/* A-posteriori bounds on the error of the measures of z against those of the
 * exact z* = (I+L)^{-1} s.  With the residual level
 *   tau = max_v |s_v - ((I+L) z)_v| / (s_v + c)
 * (the shift c >= 0 cancels in the residual because (I+L) 1 = 1), Lemma 7
 * applied to the shifted system gives |z'- z*'| <= tau z*' entrywise
 * (z' = z + c), hence |z_v - z*_v| <= b_v = tau (z_v + c) / (1 - tau) when
 * tau < 1.  Each bound adds up, term by term, the largest change of the
 * measure (Table 1 definitions) over moves |e_v| <= b_v:
 *   C: sum 2|z_v| b_v + b_v^2        I: sum 2|z_v - s_v| b_v + b_v^2
 *   P: sum 2|z_v - m| b_v + b_v^2    (the centred values sum to zero, so the
 *      mean's move drops out of the first-order term)
 *   D: sum over edges a_ij (2|z_i - z_j|(b_i + b_j) + (b_i + b_j)^2)
 *   mean: mean b.
 * Valid for any z, certified or not; a solve certified at (eps, c, sigma) has
 * tau <= eps' = sigma eps / (c + sigma).  tau is infinite where some
 * s_v + c = 0 (c = 0 with a zero opinion).  tau >= 1: every bound is +inf.
 * s, z: device [n].  out: [host] the measures, bitwise equal to fj_metrics.
 * bound: [host] the bounds in the same fields.  tau: [host] or NULL.
 * Workspace: fj_metrics_workspace_bytes.  Synchronizes `stream`. */
fj_status fj_metrics_bounds(const fj_graph* g, const double* s, const double* z, double c, fj_metrics_out* out,
                            fj_metrics_out* bound, double* tau, void* ws, size_t ws_bytes, void* stream);

size_t fj_stress_workspace_bytes(const fj_graph* g);

/* Stress of Sec. 3.4 for every node: stress_i = (z_i - s_i)^2 + sum_j a_ij (z_i - z_j)^2
 * over row i of A (the nodes i listens to), in FP64.
 * s, z: device [n].  stress: device [n] output, or NULL to return the total only.
 * total: [host] sum_i stress_i in a fixed order (bitwise reproducible).  With D
 * as fj_metrics reports it, the total equals I + 2D on an undirected graph (every
 * edge is in two rows) and I + D on a directed one; the text of Sec. 3.4 states
 * I + D for both.  Synchronizes `stream`. */
fj_status fj_stress(const fj_graph* g, const double* s, const double* z, double* stress, double* total,
                    void* ws, size_t ws_bytes, void* stream);

/* FP64 certificate of an arbitrary z: max_v |s_v - ((I+L) z)_v| / (eps' (s_v + c)).
 * out_max_ratio: [host].  Synchronizes `stream`.  Uses the metrics workspace. */
fj_status fj_certify(const fj_graph* g, const double* s, const double* z, double eps, double c,
                     double sigma, double* out_max_ratio, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- diagnostics */

/* The random-gather ceiling of the sweep's access pattern on this graph: one
 * launch over every arc of the colour-major CSR (the original CSR when the
 * graph has no colouring) that streams the column index and gathers the value
 * at it, value_bytes = 4 (the fixed-point copy the early sweeps read) or 8
 * (the FP64 estimate), four loads in flight per lane, and nothing else.  A
 * sweep of Eq. (sor1) in pull form does this plus its per-row arithmetic, so
 * its arc rate divided by this one is the fraction of the gather ceiling it
 * reaches.  One untimed launch, then `reps` (1..1000) launches timed with HIP
 * events on `stream`.  arcs_per_s: [host] out, arcs per second.
 * Synchronizes `stream`. */
size_t fj_gather_probe_workspace_bytes(const fj_graph* g);
fj_status fj_gather_probe(const fj_graph* g, int32_t value_bytes, int32_t reps, double* arcs_per_s, void* ws,
                          size_t ws_bytes, void* stream);

/* ----------------------------------------------------------- batched solve
 * Many opinion vectors and many graphs solved by one enqueued sequence that
 * never synchronizes the host (capture-safe), so a whole batch can run as one
 * hipGraph launch.  Items with k = 1 are joined into one block-diagonal graph
 * whose components stop sweeping once their own sweep is quiet; items with
 * k > 1 keep their k vectors node-major ([n][k]) so every arc reads k
 * estimates in one coalesced access.  The method per vector is the same
 * colour-ordered ImprovedBLISOR as fj_solve (FP64 sweeps), with the same
 * certificate (Lemma 7 with the shift of Alg. 2). */

typedef struct fj_batch fj_batch;

typedef struct {
    fj_graph_desc graph; /* device CSR, same rules as fj_graph_create; must outlive the batch */
    int32_t k;           /* opinion vectors on this graph, 1..64 */
} fj_batch_item_desc;

/* Bytes of batch workspace (graphs' ingest products, inputs, outputs, state). */
size_t fj_batch_workspace_bytes(const fj_batch_item_desc* items, int32_t num_items);

/* Validate and ingest every graph (as fj_graph_create with FJ_GRAPH_COLOUR).
 * opts: eps, omega, c, sigma as for fj_solve (precision and schedule ignored:
 * FP64 colour-ordered sweeps); max_refinements unused; check_every unused.
 * The sweep budget starts at 256 and is reset by fj_batch_tune.  Synchronizes. */
fj_status fj_batch_create(const fj_batch_item_desc* items, int32_t num_items, const fj_solve_opts* opts, void* ws,
                          size_t ws_bytes, void* stream, fj_batch** out);
fj_status fj_batch_destroy(fj_batch* b);

/* Device pointers, inside the batch workspace, of item i's input s ([n][k]
 * node-major, FP64) and output z (same layout).  The caller writes s there
 * before fj_solve_batched; z is valid after it. [host] out. */
fj_status fj_batch_io(const fj_batch* b, int32_t item, double** s, double** z);

/* Autotuner (synchronizes): with the inputs currently in place, solves the
 * batch once for each omega in omegas[0..n_omegas) and keeps, per item group
 * (undirected single-vector items, directed single-vector items, each
 * multi-vector item), the one that needed the fewest sweeps; then times the
 * launch parameters at those omegas, one at a time: 64-arc chunks in flight
 * per light tile of the single-vector union (2, 4 or 8) and value rows in
 * flight per wave of the multi-vector rows (4, 8 or 16), which leave the sums
 * and the result unchanged.  The choice is kept for the life of the process under the
 * batch's shape (eps, c, sigma; per group the item count and the base-2
 * magnitude of nodes and arcs; per multi-vector item k, nodes, arcs and
 * direction): a later batch of the same shape takes it without timing (one
 * solve still measures the sweeps its inputs need).  The sweep budget is the
 * sweeps needed plus max(4, 25%), and the launch sequence is recorded into a
 * hipGraph that fj_solve_batched replays, with the single-vector union and
 * the multi-vector items as two concurrent branches (independent systems;
 * each branch decides its own convergence, so the result is the same as
 * the one-stream sequence's, bit for bit).  [host] omegas.
 * FJ_ERR_NOT_CONVERGED if an item needs more than 512 sweeps for every
 * candidate. */
fj_status fj_batch_tune(fj_batch* b, const double* omegas, int32_t n_omegas, void* stream);

/* Forget every shape kept by fj_batch_tune in this process. */
void fj_batch_tune_cache_clear(void);

/* Caller-owned inputs and outputs: s[i] and z[i] ([host] arrays of num_items
 * device pointers) hold item i's opinions and receive its equilibrium, n_i x k_i
 * doubles node-major, in place of the workspace buffers of fj_batch_io.  Every
 * later solve copies s[i] in at its start and writes z[i] at its end, inside
 * the same enqueued sequence (a recorded hipGraph is recorded again with the
 * copies).  The buffers must stay valid while bound.  s = z = NULL unbinds.
 * Synchronizes `stream`. */
fj_status fj_batch_bind(fj_batch* b, const double* const* s, double* const* z, void* stream);

/* After fj_solve_batched (synchronizes): counts the items whose FP64
 * certificate failed, normally because their inputs need more sweeps than
 * the budget recorded by fj_batch_tune.  With extra_sweeps > 0 those items
 * sweep on from their current estimates (Lemma 4: any estimate is a valid
 * start) for up to extra_sweeps more sweeps, the results of every item are
 * recomputed (and copied to the bound outputs), and they are counted again.
 * uncertified: [host] out.  stats_dev, metrics_dev: device, as for
 * fj_solve_batched, or NULL; they receive the items' stats and measures after
 * the check (and its continuation).  FJ_OK when every item is certified,
 * else FJ_ERR_NOT_CONVERGED. */
fj_status fj_batch_check(fj_batch* b, int32_t extra_sweeps, int32_t* uncertified, fj_solve_stats* stats_dev,
                         fj_metrics_out* metrics_dev, void* stream);

typedef struct {
    double omega;         /* relaxation factor of the last item group */
    double omega_undirected; /* chosen for the undirected single-vector items (0 if none) */
    double omega_directed;   /* chosen for the directed single-vector items (0 if none) */
    double omega_multi;      /* chosen for the first multi-vector item (0 if none) */
    int32_t sweep_budget; /* sweeps recorded per solve */
    int32_t graph_nodes;  /* kernel launches in the recorded hipGraph (0 if none) */
    int32_t num_colours;  /* most colour classes over the items */
    double tune_ms[16];   /* measured time per candidate omega (0 when the shape was known) */
    int32_t union_chunks_in_flight; /* launch parameter chosen for the single-vector union */
    int32_t multi_arcs_in_flight;   /* launch parameter chosen for the multi-vector items */
    int32_t cache_hit;    /* 1: the last fj_batch_tune took a shape kept from an earlier batch */
    int32_t bound;        /* 1: inputs and outputs are caller-bound (fj_batch_bind) */
} fj_batch_info;
fj_status fj_batch_get_info(const fj_batch* b, fj_batch_info* out);

/* Set the launch parameters fj_batch_tune picks by hand: 64-arc chunks in
 * flight per light tile of the union (union_chunks: 2, 4 or 8) and arcs in
 * flight per wave of the multi-vector rows (multi_arcs: 4, 8 or 16); 0 leaves
 * a parameter as it is.
 * Neither changes the sums, so results stay bit for bit the same.  A recorded
 * hipGraph is recorded again with them.  Errors: FJ_ERR_INVALID_ARGUMENT,
 * FJ_ERR_HIP. */
fj_status fj_batch_set_launch(fj_batch* b, int32_t union_chunks, int32_t multi_arcs);

/* Set the relaxation factor per item group by hand (each in (0,2); a value <= 0
 * leaves that group unchanged) and drop any recorded hipGraph, so that
 * fj_solve_batched enqueues the kernels directly with the current budget. */
fj_status fj_batch_set_omegas(fj_batch* b, double omega_undirected, double omega_directed, double omega_multi);

/* Solve every item.  Enqueues only (never synchronizes; uses no host memory):
 * the recorded hipGraph if fj_batch_tune ran, else the kernels directly.
 * stats_dev: device [num_items] or NULL; per item rounds = sweeps used,
 * certified, max_ratio (over its k vectors), edge_visits = arcs whose value
 * was gathered (a multi-vector item: for each vector, its arcs times the
 * sweeps until it went quiet); other fields 0.
 * metrics_dev: device [sum of k] or NULL, item-major then vector. */
fj_status fj_solve_batched(fj_batch* b, fj_solve_stats* stats_dev, fj_metrics_out* metrics_dev, void* stream);

/* ------------------------------------------------------- learned warm start
 * Not part of the paper's method.  A two-layer message-passing network
 * proposes a starting estimate z0; by Lemma 4 any start is valid and by
 * Lemma 7 the same residual certificate decides the result, so passing z0 as
 * fj_solve_opts.z0 only changes how long the sweeps run.  Network (hidden
 * width 64, BF16 operands on MFMA, FP32 accumulation):
 *   ns = nbr(s), z1 = (s + d ns) / (1 + d)  (one step of Eq. (1) from s)
 *   X0 = [s, ns, z1, log1p d, 1/(1+d), mean s, 1, 0]
 *   H1 = relu(X0 W1 + b1),  P = H1 Wp,  M = nbr(P)
 *   H2 = relu([H1 | M] W2 + b2)
 *   z0 = min s + (max s - min s) sigmoid(H2 u + c0),  nbr(x)_v = sum_j a_vj x_j / d_v
 * Layer 1's message is the opinion, layer 2's the 16-wide P.
 * params: device FP32 [fj_wsnet_param_count()] = W1 (8x64 row-major), b1 (64),
 * Wp (64x16), W2 (80x64), b2 (64), u (64), c0 (1).  The graph must come from
 * fj_graph_create (any flags).  Training minimises the mean over nodes of
 * w_v (z0_v - z_v)^2 against a target z (normally a tighter solve of the same
 * problem), w_v = 1 / (z_v + rel_floor)^2 when rel_floor > 0 (the
 * certificate is relative), else 1. */
int32_t fj_wsnet_param_count(void);
/* training != 0: room for the backward pass as well. */
size_t fj_wsnet_workspace_bytes(const fj_graph* g, int32_t training);
/* z0: device [n] out.  s: device [n]. */
fj_status fj_wsnet_forward(const fj_graph* g, const double* s, const float* params, double* z0, void* ws,
                           size_t ws_bytes, void* stream);
/* fj_wsnet_forward with its four stages timed by HIP events on `stream`, for
 * measuring the network against its rooflines.  stage_ms: [host] 4 out: the
 * statistics and the gather of s (ns), k_net_l1 (features, layer 1 and P on
 * MFMA tiles), the gather of P (M), k_net_l2 (layer 1 again, layer 2 and the
 * readout on MFMA tiles).  Synchronizes the stream.  Errors as
 * fj_wsnet_forward, and FJ_ERR_HIP if an event call fails. */
fj_status fj_wsnet_forward_timed(const fj_graph* g, const double* s, const float* params, double* z0, void* ws,
                                 size_t ws_bytes, double* stage_ms, void* stream);
/* grad: device [param_count] out; loss: device scalar out (the weighted mean squared error). */
fj_status fj_wsnet_grad(const fj_graph* g, const double* s, const double* z_target, const float* params,
                        double rel_floor, float* grad, float* loss, void* ws, size_t ws_bytes, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on params; adam_m/adam_v:
 * device [param_count] moment buffers (zero before step 1); step >= 1. */
fj_status fj_wsnet_train_step(const fj_graph* g, const double* s, const double* z_target, float* params,
                              float* adam_m, float* adam_v, int32_t step, float lr, double rel_floor, float* loss,
                              void* ws, size_t ws_bytes, void* stream);

/* `steps` synchronous applications of the FJ update of Eq. (1),
 * z_i <- (s_i + sum_j a_ij z_j) / (1 + d_i), in place on z (device [n]).
 * The untrained warm-start control. */
size_t fj_jacobi_workspace_bytes(const fj_graph* g);
fj_status fj_jacobi_steps(const fj_graph* g, const double* s, double* z, int32_t steps, void* ws, size_t ws_bytes,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FJ_H */
