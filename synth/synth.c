/*
 * Seeded synthetic inputs: graphs in CSR form and internal-opinion vectors.
 *
 * This module holds none of the Friedkin-Johnsen arithmetic.  It only draws
 * random graphs and random opinion vectors, so both the FP64 oracle and the
 * HIP library can be fed identical inputs.  Every random number comes from
 * splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), keyed by (seed, stream, index) so results do not
 * depend on the number of threads.
 *
 * CSR convention: row i lists the nodes j with a_ij > 0, i.e. the nodes that
 * node i listens to (the sum in the FJ update of Sec. 3.3, Eq. (1)).  Rows are
 * sorted by column, without self-loops or duplicates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
/* counter-based draw: the k-th 64-bit word of stream (seed, stream) */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t k) {
    return mix64(mix64(seed * 0x100000001b3ULL + stream) ^ (k * 0xd1b54a32d192ed03ULL));
}
static inline double to_u01(uint64_t x) { /* (0,1): 53 bits, never 0 */
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------------- opinions */
enum { S_UNIFORM = 0, S_BETA = 1, S_BIMODAL = 2, S_EXP = 3, S_PARETO = 4 };

/* k-th smallest (1-based) of m uniforms: a Beta(k, m+1-k) variate */
static double order_stat(uint64_t seed, uint64_t i, int k, int m) {
    double u[32];
    for (int t = 0; t < m; ++t) u[t] = to_u01(draw(seed, 1000 + t, i));
    for (int a = 1; a < m; ++a) { /* insertion sort, m <= 32 */
        double x = u[a]; int b = a - 1;
        while (b >= 0 && u[b] > x) { u[b + 1] = u[b]; --b; }
        u[b + 1] = x;
    }
    return u[k - 1];
}

/* kind: S_UNIFORM U[0,1]; S_BETA Beta(a,b) (integers a,b>=1, a+b<=33);
 * S_BIMODAL 0.5 Beta(a,b) + 0.5 Beta(b,a); S_EXP x_min + Exp(1), x_min = p1,
 * divided by the max; S_PARETO x_min u^(-1/(alpha-1)), alpha = p1, divided by
 * the max.  Returns 0 on success. */
int synth_opinions(int64_t n, int kind, int a, int b, double p1, uint64_t seed, double* s) {
    if (n < 0 || !s) return 1;
    if ((kind == S_BETA || kind == S_BIMODAL) && (a < 1 || b < 1 || a + b - 1 > 32)) return 1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x;
        switch (kind) {
        case S_UNIFORM: x = to_u01(draw(seed, 1, (uint64_t)i)); break;
        case S_BETA: x = order_stat(seed, (uint64_t)i, a, a + b - 1); break;
        case S_BIMODAL: {
            int left = (draw(seed, 2, (uint64_t)i) >> 63) == 0;
            x = left ? order_stat(seed, (uint64_t)i, a, a + b - 1)
                     : order_stat(seed, (uint64_t)i, b, a + b - 1);
            break;
        }
        case S_EXP: x = p1 - log(to_u01(draw(seed, 3, (uint64_t)i))); break;
        case S_PARETO: x = pow(to_u01(draw(seed, 4, (uint64_t)i)), -1.0 / (p1 - 1.0)); break;
        default: x = 0.0;
        }
        s[i] = x;
    }
    if (kind == S_EXP || kind == S_PARETO) {
        double mx = 0.0;
        for (int64_t i = 0; i < n; ++i) if (s[i] > mx) mx = s[i];
        if (mx > 0) for (int64_t i = 0; i < n; ++i) s[i] /= mx;
    }
    return 0;
}

/* ----------------------------------------------------------- CSR assembly */
static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}
static void sort_row(int32_t* v, int64_t len) {
    if (len > 48) { qsort(v, (size_t)len, sizeof(int32_t), cmp_i32); return; }
    for (int64_t a = 1; a < len; ++a) {
        int32_t x = v[a]; int64_t b = a - 1;
        while (b >= 0 && v[b] > x) { v[b + 1] = v[b]; --b; }
        v[b + 1] = x;
    }
}
/* Sort every row, drop duplicates, compact in place.  cnt[i] = entries in row
 * i of the scattered layout starting at off[i]; rebuilds row_ptr. */
static int64_t finish_csr(int64_t n, const int64_t* off, int64_t* cnt, int32_t* col, int32_t* row_ptr) {
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
        int32_t* v = col + off[i];
        int64_t len = cnt[i];
        sort_row(v, len);
        int64_t k = 0;
        for (int64_t t = 0; t < len; ++t)
            if (k == 0 || v[t] != v[k - 1]) v[k++] = v[t];
        cnt[i] = k;
    }
    int64_t pos = 0;
    for (int64_t i = 0; i < n; ++i) {
        row_ptr[i] = (int32_t)pos;
        if (pos != off[i]) memmove(col + pos, col + off[i], (size_t)cnt[i] * sizeof(int32_t));
        pos += cnt[i];
    }
    row_ptr[n] = (int32_t)pos;
    return pos;
}

/* --------------------------------------------------------- Barabasi-Albert */
/* BA(n, m): seed clique on m+1 nodes, then node t attaches to m distinct
 * earlier nodes chosen with probability proportional to current degree (the
 * repeated-endpoint list).  Undirected, unit weights; stored both ways.
 * cap = capacity of col (needs >= (m+1)m + 2(n-m-1)m).  Returns nnz or -1. */
int64_t synth_ba(int64_t n, int m, uint64_t seed, int32_t* row_ptr, int32_t* col, int64_t cap) {
    if (m < 1 || n < m + 1) return -1;
    int64_t E = (int64_t)(m + 1) * m / 2 + (n - m - 1) * (int64_t)m;
    if (cap < 2 * E) return -1;
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * E);
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * E);
    int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * 2 * E);
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * m);
    if (!eu || !ev || !ends || !pick) { free(eu); free(ev); free(ends); free(pick); return -1; }
    int64_t ne = 0, nend = 0;
    for (int a = 0; a <= m; ++a)
        for (int b = a + 1; b <= m; ++b) {
            eu[ne] = a; ev[ne] = b; ++ne; ends[nend++] = a; ends[nend++] = b;
        }
    uint64_t k = 0;
    for (int64_t t = m + 1; t < n; ++t) {
        int got = 0;
        while (got < m) {
            int32_t c = ends[draw(seed, 7, k++) % (uint64_t)nend];
            int dup = 0;
            for (int q = 0; q < got; ++q) dup |= (pick[q] == c);
            if (!dup) pick[got++] = c;
        }
        for (int q = 0; q < m; ++q) {
            eu[ne] = (int32_t)t; ev[ne] = pick[q]; ++ne;
            ends[nend++] = (int32_t)t; ends[nend++] = pick[q];
        }
    }
    int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    for (int64_t e = 0; e < E; ++e) { cnt[eu[e]]++; cnt[ev[e]]++; }
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    memset(cnt, 0, sizeof(int64_t) * n);
    for (int64_t e = 0; e < E; ++e) {
        col[off[eu[e]] + cnt[eu[e]]++] = ev[e];
        col[off[ev[e]] + cnt[ev[e]]++] = eu[e];
    }
    int64_t nnz = finish_csr(n, off, cnt, col, row_ptr);
    free(eu); free(ev); free(ends); free(pick); free(cnt); free(off);
    return nnz;
}

/* -------------------------------------------------------------- Chung-Lu */
/* Expected-degree weights w_i = kappa (i + i0)^(-alpha), alpha = 1/(gamma-1):
 * a power law with exponent gamma in index order (node 0 heaviest).  i0 is
 * set so that w_0 equals the cutoff w_max and kappa so that sum_i w_i = total
 * (integral approximation for i0, exact sum for kappa). */
static void cl_weights(int64_t n, double gamma, double total, double wmax, double* w) {
    double alpha = 1.0 / (gamma - 1.0);
    double target = total / wmax, lo = 1e-6, hi = 1e12;
    for (int it = 0; it < 200; ++it) { /* f(i0) = i0^alpha * int_{-1/2}^{n-1/2} (x+i0)^-alpha dx */
        double i0 = sqrt(lo * hi), f;
        double A = i0 - 0.5 > 1e-9 ? i0 - 0.5 : 1e-9, B = n - 0.5 + i0;
        if (fabs(alpha - 1.0) < 1e-12) f = pow(i0, alpha) * log(B / A);
        else f = pow(i0, alpha) * (pow(B, 1 - alpha) - pow(A, 1 - alpha)) / (1 - alpha);
        if (f < target) lo = i0; else hi = i0;
    }
    double i0 = sqrt(lo * hi), sum = 0.0;
    for (int64_t i = 0; i < n; ++i) { w[i] = pow((double)i + i0, -alpha); sum += w[i]; }
    double kappa = total / sum;
    for (int64_t i = 0; i < n; ++i) w[i] *= kappa;
}

/* Vose alias table for sampling index i with probability w_i / sum w */
typedef struct { double* prob; int32_t* alias; int64_t n; } alias_t;
static int alias_build(const double* w, int64_t n, alias_t* t) {
    t->n = n;
    t->prob = (double*)malloc(sizeof(double) * n);
    t->alias = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* small = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* large = (int32_t*)malloc(sizeof(int32_t) * n);
    if (!t->prob || !t->alias || !small || !large) return 1;
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += w[i];
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        t->prob[i] = w[i] * (double)n / sum;
        t->alias[i] = (int32_t)i;
        if (t->prob[i] < 1.0) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
    }
    while (ns > 0 && nl > 0) {
        int32_t a = small[--ns], g = large[nl - 1];
        t->alias[a] = g;
        t->prob[g] = (t->prob[g] + t->prob[a]) - 1.0;
        if (t->prob[g] < 1.0) { --nl; small[ns++] = g; }
    }
    while (nl > 0) t->prob[large[--nl]] = 1.0;
    while (ns > 0) t->prob[small[--ns]] = 1.0;
    free(small); free(large);
    return 0;
}
static inline int32_t alias_draw(const alias_t* t, uint64_t x) {
    uint64_t i = (uint64_t)(((unsigned __int128)x * (uint64_t)t->n) >> 64);
    double u = to_u01(mix64(x ^ 0x5bd1e9955bd1e995ULL));
    return u < t->prob[i] ? (int32_t)i : t->alias[i];
}

/* Chung-Lu graph with expected degrees following a power law.
 *   undirected=1: M edge samples {u,v}, u and v drawn independently with
 *     probability proportional to w; stored both ways (so nnz ~ 2M).
 *   undirected=0: M arc samples: row u (the listener) drawn proportional to
 *     w in index order, column v proportional to w under an independent random
 *     permutation of the node labels (out- and in-degrees follow the same law,
 *     uncorrelated).
 * Self-loops and duplicates are dropped, so nnz is slightly below the target.
 * wmax <= 0 selects the structural cutoff sqrt(total).  weighted=1 gives each
 * stored arc a weight U[lo, hi] from a hash of (seed, endpoints); undirected
 * weights are symmetric.  col must hold 2M (undirected) or M (directed).
 * Returns nnz or -1. */
int64_t synth_chung_lu(int64_t n, int64_t M, double gamma, double wmax, int undirected,
                       uint64_t seed, int32_t* row_ptr, int32_t* col, int64_t cap,
                       int weighted, double wlo, double whi, float* wout) {
    if (n < 2 || M < 1 || gamma <= 1.0) return -1;
    int64_t slots = undirected ? 2 * M : M;
    if (cap < slots) return -1;
    double total = undirected ? 2.0 * (double)M : (double)M;
    if (wmax <= 0) wmax = sqrt(total);
    double* w = (double*)malloc(sizeof(double) * n);
    int32_t* perm = NULL;
    alias_t tab;
    if (!w) return -1;
    cl_weights(n, gamma, total, wmax, w);
    if (alias_build(w, n, &tab)) return -1;
    free(w);
    if (!undirected) { /* Fisher-Yates permutation of labels for the in-endpoints */
        perm = (int32_t*)malloc(sizeof(int32_t) * n);
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; --i) {
            int64_t j = (int64_t)(((unsigned __int128)draw(seed, 11, (uint64_t)i) * (uint64_t)(i + 1)) >> 64);
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }
    int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    /* pass 1: counts (samples regenerated in pass 2 from the same counters) */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < M; ++e) {
        int32_t u = alias_draw(&tab, draw(seed, 12, (uint64_t)e));
        int32_t v = alias_draw(&tab, draw(seed, 13, (uint64_t)e));
        if (!undirected) v = perm[v];
        if (u == v) continue;
        #pragma omp atomic
        cnt[u]++;
        if (undirected) {
            #pragma omp atomic
            cnt[v]++;
        }
    }
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    memset(cnt, 0, sizeof(int64_t) * n);
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < M; ++e) {
        int32_t u = alias_draw(&tab, draw(seed, 12, (uint64_t)e));
        int32_t v = alias_draw(&tab, draw(seed, 13, (uint64_t)e));
        if (!undirected) v = perm[v];
        if (u == v) continue;
        int64_t p;
        #pragma omp atomic capture
        p = cnt[u]++;
        col[off[u] + p] = v;
        if (undirected) {
            #pragma omp atomic capture
            p = cnt[v]++;
            col[off[v] + p] = u;
        }
    }
    int64_t nnz = finish_csr(n, off, cnt, col, row_ptr);
    if (weighted && wout) {
        #pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                uint64_t a = (uint64_t)i, b = (uint64_t)col[k];
                if (undirected && a > b) { uint64_t t = a; a = b; b = t; }
                double u = to_u01(draw(seed, 14, (a << 32) | b));
                wout[k] = (float)(wlo + (whi - wlo) * u);
            }
    }
    free(cnt); free(off); free(tab.prob); free(tab.alias); free(perm);
    return nnz;
}
