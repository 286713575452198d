"""FP64 CPU oracle for the Friedkin-Johnsen equilibrium z = (I+L)^{-1} s.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and never imports it.

What it computes (arXiv 2507.14864):
  * ``dense_solve``      - the definition, z = (I+L)^{-1} s (Lemma 1), by LU
                           (numpy.linalg.solve) for small graphs;
  * ``exact``            - the same z to ||s-(I+L)z||_inf <= 1e-12 by Jacobi-PCG
                           (undirected) or Gauss-Seidel (directed, Eq. (gauss)),
                           which bounds |z - z_exact| entrywise by the same
                           number because (I+L)^{-1} is nonnegative and
                           row-stochastic (Sec. 3.3);
  * ``push``             - ImprovedBLISOR (Alg. 2 around Alg. 3; Alg. 1 when
                           omega = 1), sequential FIFO, FP64;
  * ``metrics``          - P, D, I, C of Table 1, compensated FP64 sums;
  * ``metrics_bounds``   - a-posteriori bounds on those measures' error from
                           the residual level, by Lemma 7;
  * ``certificate``      - max_v |r_v| / h_v for a candidate z, the stopping
                           rule of Alg. 3 with the shift of Alg. 2 (Lemma 7);
  * ``mpnn``             - the warm-start network's forward/backward in FP64.
"""
import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_threads.restype = i32
        lib.oracle_degrees.argtypes = [i64, vp, vp, vp]
        lib.oracle_transpose.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_residual.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_cg.argtypes = [i64, vp, vp, vp, vp, vp, dbl, i32]
        lib.oracle_cg.restype = i32
        lib.oracle_gs.argtypes = [i64, vp, vp, vp, vp, vp, dbl, i32]
        lib.oracle_gs.restype = i32
        lib.oracle_push.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, vp, i64, i64, vp, vp, vp]
        lib.oracle_push.restype = i32
        lib.oracle_metrics.argtypes = [i64, vp, vp, vp, i32, vp, vp, vp]
        _LIB = lib
    return _LIB


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.float32)
    return rp, col, w


def threads() -> int:
    """OpenMP threads the oracle's parallel loops (residual, CG) use."""
    return int(_lib().oracle_threads())


def degrees(g) -> np.ndarray:
    """d_i = sum_j a_ij (Sec. 3.2)."""
    rp, col, w = _graph_arrays(g)
    d = np.empty(g.n, dtype=np.float64)
    _lib().oracle_degrees(g.n, _p(rp), _p(w), _p(d))
    return d


def transpose(g):
    """CSR of A^T: row v lists u with a_uv > 0."""
    rp, col, w = _graph_arrays(g)
    trp = np.empty(g.n + 1, dtype=np.int32)
    tcol = np.empty(max(g.nnz, 1), dtype=np.int32)
    tw = np.empty(max(g.nnz, 1), dtype=np.float32)
    _lib().oracle_transpose(g.n, _p(rp), _p(col), _p(w), _p(trp), _p(tcol), _p(tw))
    return trp, tcol[:g.nnz], tw[:g.nnz]


def residual(g, b: np.ndarray, z: np.ndarray) -> np.ndarray:
    """r = b - (I+L) z in FP64 (Lemma 4: z_exact - z = (I+L)^{-1} r)."""
    rp, col, w = _graph_arrays(g)
    b = np.ascontiguousarray(b, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    r = np.empty(g.n, dtype=np.float64)
    _lib().oracle_residual(g.n, _p(rp), _p(col), _p(w), _p(b), _p(z), _p(r))
    return r


def dense_matrix(g) -> np.ndarray:
    """I + L = I + D - A as a dense FP64 matrix (Sec. 3.2)."""
    n = g.n
    M = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for k in range(int(g.row_ptr[i]), int(g.row_ptr[i + 1])):
            j = int(g.col[k])
            a = 1.0 if g.w is None else float(g.w[k])
            M[i, j] -= a
            M[i, i] += a
    M[np.diag_indices(n)] += 1.0
    return M


def dense_solve(g, s: np.ndarray) -> np.ndarray:
    """z = (I+L)^{-1} s by LU with partial pivoting (Lemma 1)."""
    return np.linalg.solve(dense_matrix(g), np.asarray(s, dtype=np.float64))


def cg(g, s, tol: float = 1e-12, maxit: int = 100000, z0=None):
    """Jacobi-PCG on (I+L) z = s, undirected only.  Returns (z, iterations)."""
    if g.directed:
        raise ValueError("CG needs a symmetric I+L; use gs() for directed graphs")
    rp, col, w = _graph_arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.zeros(g.n) if z0 is None else np.array(z0, dtype=np.float64)
    it = _lib().oracle_cg(g.n, _p(rp), _p(col), _p(w), _p(s), _p(z), tol, maxit)
    if it < 0:
        raise RuntimeError("oracle CG did not reach the tolerance")
    return z, it


def gs(g, s, tol: float = 1e-12, maxsweeps: int = 100000, z0=None):
    """Natural-order Gauss-Seidel (Eq. (gauss)).  Returns (z, sweeps)."""
    rp, col, w = _graph_arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.zeros(g.n) if z0 is None else np.array(z0, dtype=np.float64)
    sw = _lib().oracle_gs(g.n, _p(rp), _p(col), _p(w), _p(s), _p(z), tol, maxsweeps)
    if sw < 0:
        raise RuntimeError("oracle Gauss-Seidel did not reach the tolerance")
    return z, sw


def exact(g, s, tol: float = 1e-12) -> np.ndarray:
    """z = (I+L)^{-1} s: dense LU for n <= 4096, else PCG (undirected) or
    Gauss-Seidel (directed) until ||s - (I+L) z||_inf <= tol."""
    if g.n <= 4096:
        return dense_solve(g, s)
    if g.directed:
        return gs(g, s, tol)[0]
    return cg(g, s, tol)[0]


def push(g, s, eps: float, sigma: float = 1e-5, c: float = 1e-5, omega: float = 1.0,
         z0=None, max_pops: int = 0, max_edge_visits: int = 0):
    """Sequential ImprovedBLISOR (Alg. 2 + Alg. 3).

    Returns dict(z=zhat, r=tracked residual of the shifted system, pops,
    edge_visits, capped, diverged)."""
    rp, col, w = _graph_arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    zz = None if z0 is None else np.ascontiguousarray(z0, dtype=np.float64)
    z = np.empty(g.n)
    r = np.empty(g.n)
    st = np.zeros(2, dtype=np.int64)
    capped = _lib().oracle_push(g.n, _p(rp), _p(col), _p(w), _p(s), eps, sigma, c, omega,
                                _p(zz), max_pops, max_edge_visits, _p(z), _p(r), _p(st))
    return dict(z=z, r=r, pops=int(st[0]), edge_visits=int(st[1]), capped=capped == 1,
                diverged=capped == 2)


def metrics(g, s, z) -> dict:
    """Table 1: P, D, I, C (+ mean of z), compensated FP64."""
    rp, col, w = _graph_arrays(g)
    s = np.ascontiguousarray(s, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(5)
    _lib().oracle_metrics(g.n, _p(rp), _p(col), _p(w), 1 if g.directed else 0, _p(s), _p(z), _p(out))
    return dict(P=out[0], D=out[1], I=out[2], C=out[3], mean=out[4])


def jacobi_spectral_radius(g) -> float:
    """mu = rho((I+D)^{-1} A), the quantity Eq. (optimal-omega) takes (Sec. 5.2).

    n <= 2000: every eigenvalue of the dense matrix (LAPACK).  Larger graphs:
    scipy's ARPACK for the one eigenvalue wanted.  Undirected graphs use the
    similar symmetric matrix (I+D)^{-1/2} A (I+D)^{-1/2} and its largest
    algebraic eigenvalue (Lanczos), which is mu by Perron-Frobenius (the
    matrix is nonnegative); directed graphs the largest-magnitude eigenvalue
    of (I+D)^{-1} A (Arnoldi).  Both start from the Perron vector of a
    regular graph ((I+D)^{1/2} 1 and 1)."""
    d = degrees(g)
    if g.n == 0:
        return 0.0
    if g.n <= 2000:
        M = dense_matrix(g)  # I + L
        A = np.diag(1.0 + d) - M
        J = A / (1.0 + d)[:, None]
        return float(np.max(np.abs(np.linalg.eigvals(J))))
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    w = np.ones(g.nnz) if g.w is None else g.w.astype(np.float64)
    A = sp.csr_matrix((w, g.col, g.row_ptr), shape=(g.n, g.n))
    if not g.directed:
        q = 1.0 / np.sqrt(1.0 + d)
        S = sp.diags(q) @ A @ sp.diags(q)
        vals = spla.eigsh(S, k=1, which="LA", v0=np.sqrt(1.0 + d), tol=1e-13, maxiter=100000,
                          return_eigenvectors=False)
        return float(vals[0])
    J = sp.diags(1.0 / (1.0 + d)) @ A
    vals = spla.eigs(J, k=1, which="LM", v0=np.ones(g.n), tol=1e-13, maxiter=100000,
                     return_eigenvectors=False)
    return float(np.max(np.abs(vals)))


def optimal_omega(mu: float) -> float:
    """Eq. (optimal-omega): 1 + (mu / (1 + sqrt(1 - mu^2)))^2."""
    return 1.0 + (mu / (1.0 + np.sqrt(1.0 - mu * mu))) ** 2


def stress(g, s, z) -> np.ndarray:
    """Stress of every node (Sec. 3.4): (z_i - s_i)^2 + sum_{j in N_i} a_ij (z_i - z_j)^2,
    N_i being the nodes listed in row i of A.  Plain per-node loops over the rows,
    math.fsum per row."""
    import math
    s = np.asarray(s, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = np.empty(g.n)
    for i in range(g.n):
        terms = [(z[i] - s[i]) ** 2]
        for k in range(int(g.row_ptr[i]), int(g.row_ptr[i + 1])):
            a = 1.0 if g.w is None else float(g.w[k])
            terms.append(a * (z[i] - z[g.col[k]]) ** 2)
        out[i] = math.fsum(terms)
    return out


def metrics_bounds(g, s, z, c: float = 1e-5):
    """A-posteriori bounds on |M(z) - M(z_exact)| for the Table 1 measures.

    Residual level tau = max_v |r_v| / (s_v + c) with r = s - (I+L) z; the
    shift cancels in r because (I+L) 1 = 1.  Lemma 7 on the shifted system
    gives |z' - z_exact'| <= tau z_exact' entrywise, so z_exact' <= z' / (1 - tau)
    and |z_v - z_exact_v| <= b_v = tau (z_v + c) / (1 - tau) for tau < 1.  Each
    measure's bound adds up, term by term, the largest change that moves
    e_v with |e_v| <= b_v can cause: (x + e)^2 - x^2 = 2 x e + e^2, and
    z_i - z_j moves by at most b_i + b_j.  For P the centred values sum to
    zero, so the mean's move drops out of the first-order term and only
    lowers the second-order one: |dP| <= sum 2|z_v - m| b_v + b_v^2.  The mean
    moves by at most mean(b).  Returns (bounds dict with P, D, I, C, mean;
    tau); infinite bounds when tau >= 1.  math.fsum for every sum."""
    import math
    s = np.asarray(s, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = g.n
    if n == 0:
        return dict(P=0.0, D=0.0, I=0.0, C=0.0, mean=0.0), 0.0
    r = residual(g, s, z)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.abs(r) / (s + c)
    ratio[~np.isfinite(ratio)] = np.inf
    tau = float(np.max(ratio))
    if not tau < 1.0:
        inf = float("inf")
        return dict(P=inf, D=inf, I=inf, C=inf, mean=inf), tau
    b = tau * (z + c) / (1.0 - tau)
    m = math.fsum(z) / n
    B = math.fsum(b) / n
    C = math.fsum(2.0 * np.abs(z) * b + b * b)
    I = math.fsum(2.0 * np.abs(z - s) * b + b * b)
    P = math.fsum(2.0 * np.abs(z - m) * b + b * b)
    terms = []
    for i in range(n):
        for k in range(int(g.row_ptr[i]), int(g.row_ptr[i + 1])):
            j = int(g.col[k])
            a = 1.0 if g.w is None else float(g.w[k])
            terms.append(a * (2.0 * abs(z[i] - z[j]) * (b[i] + b[j]) + (b[i] + b[j]) ** 2))
    D = math.fsum(terms)
    if not g.directed:  # every undirected edge is stored as two arcs
        D *= 0.5
    return dict(P=P, D=D, I=I, C=C, mean=B), tau


def certificate(g, s, z, eps: float, sigma: float = 1e-5, c: float = 1e-5) -> float:
    """max_v |r_v| / h_v with r = s' - (I+L)(z + c) = s - (I+L) z and
    h = eps' (s + c), eps' = sigma eps / (c + sigma) (Alg. 2, Alg. 3).
    A value <= 1 certifies |z - z_exact| <= eps' (z_exact + c) entrywise
    (Lemma 7 with the shift of Alg. 2)."""
    r = residual(g, s, z)
    h = sigma * eps / (c + sigma) * (np.asarray(s, dtype=np.float64) + c)
    return float(np.max(np.abs(r) / h)) if g.n else 0.0


def fj_iterate(g, s, z, steps: int) -> np.ndarray:
    """`steps` synchronous applications of the FJ update, Eq. (1):
    z_i <- (s_i + sum_j a_ij z_j) / (1 + sum_j a_ij)."""
    z = np.array(z, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    d = degrees(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = np.ones(g.nnz) if g.w is None else g.w.astype(np.float64)
    for _ in range(steps):
        acc = np.bincount(rows, weights=w * z[g.col], minlength=g.n)
        z = (s + acc) / (1.0 + d)
    return z


def max_rel_error(z_est, z_true, floor: float = 1e-5) -> float:
    """max over v with z_true_v >= floor of |z_est_v - z_true_v| / z_true_v
    (the error measure of Sec. 6 restricted as in the ImprovedBLI lemma)."""
    z_est = np.asarray(z_est, dtype=np.float64)
    z_true = np.asarray(z_true, dtype=np.float64)
    m = z_true >= floor
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(z_est[m] - z_true[m]) / z_true[m]))
