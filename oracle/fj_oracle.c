/*
 * FP64 CPU oracle for the Friedkin-Johnsen (FJ) equilibrium and its measures.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP path.
 *
 * Plain, slow, obviously correct implementations, each following a passage of
 * "Efficient Algorithms for Relevant Quantities of Friedkin-Johnsen Opinion
 * Dynamics Model" (arXiv 2507.14864):
 *   - oracle_residual:  r = s - (I+L) z                      (Lemma 1, Lemma 4)
 *   - oracle_cg:        Jacobi-preconditioned CG on (I+L) z = s, undirected
 *                       graphs only (I+L symmetric positive definite, Sec. 5.2)
 *   - oracle_gs:        Gauss-Seidel sweeps on (I+L) z = s   (Eq. (gauss))
 *   - oracle_push:      ImprovedBLISOR = Alg. 2's shift around Alg. 3
 *                       (Alg. 1 when omega = 1)
 *   - oracle_metrics:   I, D, P, C of Table 1 with the mean-centred z of Sec. 3.4
 *
 * Graph convention: CSR of A, row i lists j with a_ij > 0 (node i listens to
 * node j, the sum of Eq. (1)); w == NULL means unit weights; d_i = sum_j a_ij;
 * L = D - A.  A push at v hands residual to every u with a_uv > 0 (column v of
 * A, as in the proof of Lemma 4), so the push walks CSR(A^T).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double wgt(const float* w, int64_t k) { return w ? (double)w[k] : 1.0; }

/* Neumaier-compensated summation */
typedef struct { double s, c; } ksum_t;
static inline void kadd(ksum_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double kval(const ksum_t* a) { return a->s + a->c; }

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* d_i = sum_j a_ij (Sec. 3.2; weighted form of the denominator of Eq. (1)) */
void oracle_degrees(int64_t n, const int32_t* row_ptr, const float* w, double* d) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += wgt(w, k);
        d[i] = s;
    }
}

/* CSR(A^T) by counting: row v of the result lists u with a_uv > 0 and weight a_uv. */
void oracle_transpose(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
                      int32_t* t_row_ptr, int32_t* t_col, float* t_w) {
    int64_t nnz = row_ptr[n];
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k) cnt[col[k] + 1]++;
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    for (int64_t v = 0; v <= n; ++v) t_row_ptr[v] = (int32_t)cnt[v];
    for (int64_t u = 0; u < n; ++u)
        for (int64_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k) {
            int64_t p = cnt[col[k]]++;
            t_col[p] = (int32_t)u;
            if (t_w) t_w[p] = w ? w[k] : 1.0f;
        }
    free(cnt);
}

/* r = b - (I+L) z, row by row, with L = D - A written out per arc:
 * r_i = (b_i - z_i) + sum_j a_ij (z_j - z_i), all terms in one compensated sum
 * (the differences z_j - z_i avoid the cancellation of (1+d_i) z_i against
 * sum_j a_ij z_j at hubs).  By Lemma 4, z_exact - z = (I+L)^{-1} r, and since
 * (I+L)^{-1} is nonnegative and row-stochastic (Sec. 3.3),
 * |z_exact - z| <= (I+L)^{-1}|r| <= ||r||_inf. */
void oracle_residual(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
                     const double* b, const double* z, double* r) {
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        ksum_t acc = {0.0, 0.0};
        kadd(&acc, b[i] - z[i]);
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) kadd(&acc, wgt(w, k) * (z[col[k]] - z[i]));
        r[i] = kval(&acc);
    }
}

static double inf_norm(int64_t n, const double* r) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) if (fabs(r[i]) > m) m = fabs(r[i]);
    return m;
}

/* y = (I+L) x */
static void apply_IL(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
                     const double* d, const double* x, double* y) {
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) acc += wgt(w, k) * x[col[k]];
        y[i] = (1.0 + d[i]) * x[i] - acc;
    }
}

static double dot(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    #pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned conjugate gradients for (I+L) z = s on an undirected
 * graph (I+L symmetric positive definite).  Starts from z (in/out).  Stops when
 * the recomputed residual satisfies ||s - (I+L) z||_inf <= tol.  Returns the
 * iteration count, or -1 if maxit was reached first. */
int oracle_cg(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
              const double* s, double* z, double tol, int maxit) {
    double* d = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* y = (double*)malloc(sizeof(double) * n);
    oracle_degrees(n, row_ptr, w, d);
    oracle_residual(n, row_ptr, col, w, s, z, r);
    int it = 0, done = inf_norm(n, r) <= tol;
    for (int64_t i = 0; i < n; ++i) { y[i] = r[i] / (1.0 + d[i]); p[i] = y[i]; }
    double ry = dot(n, r, y);
    int restarts = 0;
    while (!done && it < maxit) {
        apply_IL(n, row_ptr, col, w, d, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(ry / pq)) {
            /* breakdown at the rounding floor: restart from the true residual */
            oracle_residual(n, row_ptr, col, w, s, z, r);
            if (inf_norm(n, r) <= tol) { done = 1; break; }
            if (++restarts > 50) break;
            for (int64_t i = 0; i < n; ++i) { y[i] = r[i] / (1.0 + d[i]); p[i] = y[i]; }
            ry = dot(n, r, y);
            continue;
        }
        double alpha = ry / pq;
        for (int64_t i = 0; i < n; ++i) { z[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++it;
        if (it % 8 == 0 || inf_norm(n, r) <= tol) { /* guard against recurrence drift */
            oracle_residual(n, row_ptr, col, w, s, z, r);
            if (inf_norm(n, r) <= tol) { done = 1; break; }
        }
        for (int64_t i = 0; i < n; ++i) y[i] = r[i] / (1.0 + d[i]);
        double ry2 = dot(n, r, y);
        double beta = ry2 / ry;
        ry = ry2;
        for (int64_t i = 0; i < n; ++i) p[i] = y[i] + beta * p[i];
    }
    free(d); free(r); free(p); free(q); free(y);
    return done ? it : -1;
}

/* Gauss-Seidel in natural order on (I+L) z = s (Eq. (gauss) with the active set
 * equal to V): z_i <- (s_i + sum_j a_ij z_j) / (1 + d_i), newest values first.
 * Starts from z (in/out).  After every sweep the residual is recomputed and the
 * loop stops when ||s - (I+L) z||_inf <= tol.  Returns sweeps or -1. */
int oracle_gs(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
              const double* s, double* z, double tol, int maxsweeps) {
    double* r = (double*)malloc(sizeof(double) * n);
    double* d = (double*)malloc(sizeof(double) * n);
    oracle_degrees(n, row_ptr, w, d);
    oracle_residual(n, row_ptr, col, w, s, z, r);
    int sw = 0, done = inf_norm(n, r) <= tol;
    while (!done && sw < maxsweeps) {
        for (int64_t i = 0; i < n; ++i) {
            ksum_t acc = {0.0, 0.0};  /* compensated, so hub rows reach the 1e-12 residual */
            kadd(&acc, s[i]);
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) kadd(&acc, wgt(w, k) * z[col[k]]);
            z[i] = kval(&acc) / (1.0 + d[i]);
        }
        ++sw;
        oracle_residual(n, row_ptr, col, w, s, z, r);
        done = inf_norm(n, r) <= tol;
    }
    free(r); free(d);
    return done ? sw : -1;
}

/* FIFO of node ids with a membership flag: every node is queued at most
 * once, so n + 1 slots of a ring suffice. */
typedef struct { int32_t* slot; unsigned char* queued; int64_t cap, head, tail; } fifo_t;
static void fifo_admit(fifo_t* f, int32_t v) {
    if (f->queued[v]) return;
    f->slot[f->tail] = v;
    f->tail = (f->tail + 1) % f->cap;
    f->queued[v] = 1;
}
static int32_t fifo_take(fifo_t* f) {
    int32_t v = f->slot[f->head];
    f->head = (f->head + 1) % f->cap;
    f->queued[v] = 0;
    return v;
}

/* ImprovedBLISOR: the shift of Alg. 2 (ImprovedBLI) wrapped around Alg. 3
 * (BoundLocalIterSOR), as the text after Lemma 7 describes.  omega = 1 gives
 * Alg. 1 (BoundLocalIter) inside Alg. 2.
 *
 * Shifted system (Alg. 2): s' = s + c, eps' = sigma eps / (c + sigma), and the
 * threshold of node v is h_v = eps' s'_v.  The estimate starts at zhat' = 0
 * with residual r = s', and every node waits in a FIFO queue in index order.
 * A push at v moves three things, the over-relaxed Gauss-Seidel step of
 * Sec. 5.2 written on the residual:
 *   Eq. (sor1)  zhat'_v grows by omega r_v / (1 + d_v);
 *   Eq. (sor3)  each u with a_uv > 0 (u listens to v) gains a_uv times that
 *               amount in r_u;
 *   Eq. (sor2)  r_v keeps (1 - omega) of itself.
 * After the push, every node whose residual it changed (the in-neighbours of
 * v in CSR(A^T) order, then v) joins the back of the queue if its |r| exceeds
 * its threshold and it is not already waiting.  The loop ends with an empty
 * queue, so |r| <= h everywhere and Lemma 7 gives |zhat' - z'| <= eps' z';
 * the result is zhat = zhat' - c.
 *
 * Readings where the paper is terse: the threshold uses the shifted opinions
 * s' (the proof of the ImprovedBLI lemma needs h = eps' s'); weights enter
 * Eq. (sor3) as a_uv; the threshold test is strict (|r| > h).
 *
 * Optional warm start: if z0 != NULL, zhat' = z0 + c and r = s' - (I+L) zhat'
 * (valid for any zhat' by Lemma 4); the queue then holds the nodes over
 * their threshold, in index order.
 *
 * max_pops / max_edge_visits: 0 = unlimited; when a cap stops the loop early
 * the function returns 1 (not converged).  A residual that has become NaN or
 * infinite (over-relaxation diverging, which the paper does not rule out for
 * directed graphs) makes every threshold test false, so the queue drains; this
 * is reported as 2.  Otherwise 0.  out_zhat receives
 * zhat' - c, out_r (may be NULL) the tracked residual, stats (may be NULL)
 * {pops, edge visits}. */
int oracle_push(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
                const double* s, double eps, double sigma, double c, double omega,
                const double* z0, int64_t max_pops, int64_t max_edge_visits,
                double* out_zhat, double* out_r, int64_t* stats) {
    int64_t nnz = row_ptr[n];
    int32_t* t_row_ptr = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
    int32_t* t_col = (int32_t*)malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    float* t_w = (float*)malloc(sizeof(float) * (nnz ? nnz : 1));
    double* d = (double*)malloc(sizeof(double) * n);
    double* h = (double*)malloc(sizeof(double) * n);
    double* r = (double*)malloc(sizeof(double) * n);
    double* zh = (double*)malloc(sizeof(double) * n);
    fifo_t Q = {(int32_t*)malloc(sizeof(int32_t) * (n + 1)), (unsigned char*)calloc((size_t)n + 1, 1),
                n + 1, 0, 0};
    oracle_transpose(n, row_ptr, col, w, t_row_ptr, t_col, t_w);
    oracle_degrees(n, row_ptr, w, d);

    /* the shifted problem of Alg. 2 */
    const double epsp = sigma * eps / (c + sigma);
    for (int64_t v = 0; v < n; ++v) {
        r[v] = s[v] + c;  /* s'; the residual of zhat' = 0 */
        h[v] = epsp * r[v];
        zh[v] = 0.0;
    }
    if (z0) {
        for (int64_t v = 0; v < n; ++v) zh[v] = z0[v] + c;
        double* sp = (double*)malloc(sizeof(double) * n);
        memcpy(sp, r, sizeof(double) * n);
        oracle_residual(n, row_ptr, col, w, sp, zh, r);
        free(sp);
        for (int64_t v = 0; v < n; ++v)
            if (fabs(r[v]) > h[v]) fifo_admit(&Q, (int32_t)v);
    } else {
        for (int64_t v = 0; v < n; ++v) fifo_admit(&Q, (int32_t)v);
    }

    int64_t pops = 0, visits = 0;
    int capped = 0;
    while (Q.head != Q.tail) {
        if ((max_pops && pops >= max_pops) || (max_edge_visits && visits >= max_edge_visits)) {
            capped = 1;
            break;
        }
        const int32_t v = fifo_take(&Q);
        const int64_t b = t_row_ptr[v], e = t_row_ptr[v + 1];
        const double amount = omega * r[v] / (1.0 + d[v]);
        zh[v] += amount;                                              /* Eq. (sor1) */
        for (int64_t k = b; k < e; ++k) r[t_col[k]] += (double)t_w[k] * amount; /* Eq. (sor3) */
        r[v] = (1.0 - omega) * r[v];                                  /* Eq. (sor2) */
        for (int64_t k = b; k < e; ++k)
            if (fabs(r[t_col[k]]) > h[t_col[k]]) fifo_admit(&Q, t_col[k]);
        if (fabs(r[v]) > h[v]) fifo_admit(&Q, v);
        ++pops;
        visits += e - b;
    }
    int finite = 1;
    for (int64_t v = 0; v < n; ++v) {
        out_zhat[v] = zh[v] - c;
        finite &= isfinite(zh[v]) && isfinite(r[v]);
    }
    if (out_r) memcpy(out_r, r, sizeof(double) * n);
    if (stats) { stats[0] = pops; stats[1] = visits; }
    free(t_row_ptr); free(t_col); free(t_w); free(d); free(h); free(r); free(zh);
    free(Q.slot); free(Q.queued);
    return capped ? 1 : (finite ? 0 : 2);
}

/* Table 1 measures over z, with the mean-centred vector of Sec. 3.4:
 *   out[0] P = sum_i (z_i - mean)^2        (two passes: mean first)
 *   out[1] D = sum over edges (i,j) of a_ij (z_i - z_j)^2;
 *              undirected: each edge once (half the sum over stored arcs);
 *              directed: each arc once
 *   out[2] I = sum_i (z_i - s_i)^2
 *   out[3] C = sum_i z_i^2
 *   out[4] mean = sum_i z_i / n
 * All sums are Neumaier-compensated FP64. */
void oracle_metrics(int64_t n, const int32_t* row_ptr, const int32_t* col, const float* w,
                    int directed, const double* s, const double* z, double* out) {
    ksum_t sz = {0, 0}, sc = {0, 0}, si = {0, 0}, sp = {0, 0}, sd = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        kadd(&sz, z[i]);
        kadd(&sc, z[i] * z[i]);
        kadd(&si, (z[i] - s[i]) * (z[i] - s[i]));
    }
    double mean = n ? kval(&sz) / (double)n : 0.0;
    for (int64_t i = 0; i < n; ++i) kadd(&sp, (z[i] - mean) * (z[i] - mean));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double dz = z[i] - z[col[k]];
            kadd(&sd, wgt(w, k) * dz * dz);
        }
    out[0] = kval(&sp);
    out[1] = directed ? kval(&sd) : 0.5 * kval(&sd);
    out[2] = kval(&si);
    out[3] = kval(&sc);
    out[4] = mean;
}
