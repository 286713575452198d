"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here runs on a GPU.  Each test pins one oracle function to something
other than itself: a closed form derived by hand, a matrix identity stated in
Sec. 3.3, an invariant of the push (Lemma 4, Lemma 6, Lemma 7, Thm. 8), the
Gauss-Seidel formula of Eq. (gauss), or brute force on tiny graphs.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests import graphs

EPS_SIGMA_C = dict(sigma=1e-5, c=1e-5)


# ---------------------------------------------------------------- closed forms
def test_single_edge_closed_form():
    g = graphs.from_arcs(2, [(0, 1)])
    s = np.array([0.3, 0.9])
    want = np.array([(2 * s[0] + s[1]) / 3, (s[0] + 2 * s[1]) / 3])
    assert np.allclose(oracle.dense_solve(g, s), want, rtol=0, atol=1e-15)
    assert np.allclose(oracle.gs(g, s)[0], want, atol=1e-12)


@pytest.mark.parametrize("n", [2, 5, 17])
def test_complete_graph_closed_form(n):
    g = graphs.complete(n)
    s = synth.opinions(n, "uniform", 7)
    want = (s + s.sum()) / (n + 1)
    assert np.allclose(oracle.dense_solve(g, s), want, atol=1e-14)
    assert np.allclose(oracle.cg(g, s)[0], want, atol=1e-12)
    assert np.allclose(oracle.gs(g, s)[0], want, atol=1e-12)


@pytest.mark.parametrize("k", [1, 3, 40])
def test_star_closed_form(k):
    g = graphs.star(k)
    s = synth.opinions(k + 1, "uniform", 11)
    z0 = (2 * s[0] + s[1:].sum()) / (k + 2)
    want = np.concatenate([[z0], (s[1:] + z0) / 2])
    assert np.allclose(oracle.dense_solve(g, s), want, atol=1e-14)
    assert np.allclose(oracle.cg(g, s)[0], want, atol=1e-12)


@pytest.mark.parametrize("w", [1.0, 0.7, 1.3])
def test_directed_chain_closed_form(w):
    n = 9
    g = graphs.chain(n, w)
    s = synth.opinions(n, "uniform", 5)
    want = np.empty(n)
    want[-1] = s[-1]
    for i in range(n - 2, -1, -1):
        want[i] = (s[i] + np.float32(w) * want[i + 1]) / (1 + np.float32(w))
    assert np.allclose(oracle.dense_solve(g, s), want, atol=1e-14)
    assert np.allclose(oracle.gs(g, s)[0], want, atol=1e-12)
    p = oracle.push(g, s, 1e-6)
    assert oracle.max_rel_error(p["z"], want) <= 1e-6


# ------------------------------------------------ fundamental-matrix facts
@pytest.mark.parametrize("directed,weighted,seed", [(False, False, 1), (True, False, 2),
                                                    (True, True, 3), (False, True, 4)])
def test_fundamental_matrix_properties(directed, weighted, seed):
    """(I+L)^{-1} is positive, row-stochastic, and the diagonal entry is the
    largest in its column (Sec. 3.2-3.3)."""
    g = graphs.random_graph(30, 0.15, seed, directed=directed, weighted=weighted)
    Minv = np.linalg.inv(oracle.dense_matrix(g))
    assert np.all(Minv >= -1e-15)
    assert np.allclose(Minv.sum(axis=1), 1.0, atol=1e-12)
    for j in range(g.n):
        col = Minv[:, j]
        assert np.all(col[np.arange(g.n) != j] <= col[j] + 1e-15)


def test_dense_matrix_against_laplacian_definition():
    """I + D - A assembled from an explicit adjacency matrix."""
    g = graphs.random_graph(12, 0.3, 9, directed=True, weighted=True)
    A = np.zeros((g.n, g.n))
    for i in range(g.n):
        for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
            A[i, g.col[k]] = g.w[k]
    M = np.eye(g.n) + np.diag(A.sum(axis=1)) - A
    assert np.allclose(oracle.dense_matrix(g), M, atol=1e-7)


# ------------------------------------------------------------- invariants
@pytest.mark.parametrize("directed", [False, True])
def test_exact_solvers_agree_with_dense(directed):
    g = synth.chung_lu(3000, 12000, 2.3, 21, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "bimodal", 22)
    zd = oracle.dense_solve(g, s)
    if directed:
        z, _ = oracle.gs(g, s)
    else:
        z, _ = oracle.cg(g, s)
    assert np.max(np.abs(z - zd)) <= 2e-12
    # the infinity-norm certificate bounds the entrywise error (Sec. 3.3)
    r = oracle.residual(g, s, z)
    assert np.max(np.abs(z - zd)) <= np.max(np.abs(r)) + 1e-15


@pytest.mark.parametrize("directed", [False, True])
def test_constant_opinions_are_a_fixed_point(directed):
    g = synth.chung_lu(2000, 8000, 2.1, 31, directed=directed, weighted=True)
    s = np.full(g.n, 0.37)
    assert np.allclose(oracle.exact(g, s), 0.37, atol=1e-13)
    p = oracle.push(g, s, 1e-4)
    assert oracle.max_rel_error(p["z"], s) <= 1e-4


@pytest.mark.parametrize("directed", [False, True])
def test_convex_hull_and_mass(directed):
    """z is a convex combination of s (row-stochastic nonnegative inverse), and
    for undirected graphs 1^T (I+L) = 1^T gives 1^T z = 1^T s."""
    g = synth.chung_lu(2500, 10000, 2.3, 41, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "pareto", 42)
    z = oracle.exact(g, s)
    assert z.min() >= s.min() - 1e-13 and z.max() <= s.max() + 1e-13
    if not directed:
        assert abs(z.sum() - s.sum()) <= 1e-9 * s.sum()


# ---------------------------------------------------------------- the push
def _shifted_residual(g, s, z, c):
    """s' - (I+L) zhat' with s' = s + c and zhat' = z + c."""
    return oracle.residual(g, s + c, z + c)


@pytest.mark.parametrize("omega", [1.0, 1.5, 0.7])
@pytest.mark.parametrize("directed", [False, True])
def test_lemma4_invariant_at_every_stop(omega, directed):
    """Lemma 4: the tracked residual equals s' - (I+L) zhat' after any number
    of pops (the identity holds for any pushed amount)."""
    g = synth.chung_lu(400, 2000, 2.3, 51, directed=directed, weighted=True)
    s = synth.opinions(g.n, "uniform", 52)
    for pops in [1, 7, 399, 400, 401, 1234, 5000]:
        p = oracle.push(g, s, 1e-6, omega=omega, max_pops=pops, **EPS_SIGMA_C)
        assert np.max(np.abs(p["r"] - _shifted_residual(g, s, p["z"], 1e-5))) <= 1e-13


@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_undirected_mass_conservation(omega):
    """1^T r + 1^T zhat' = 1^T s' at every stop (undirected: 1^T (I+L) = 1^T;
    the r_sum bookkeeping in the proof of Thm. 5)."""
    g = synth.barabasi_albert(300, 3, 61)
    s = synth.opinions(g.n, "exp", 62)
    c = 1e-5
    for pops in [10, 300, 777, 4000]:
        p = oracle.push(g, s, 1e-5, omega=omega, max_pops=pops, **EPS_SIGMA_C)
        assert abs(p["r"].sum() + (p["z"] + c).sum() - (s + c).sum()) <= 1e-11


@pytest.mark.parametrize("omega", [1.0, 1.3, 1.8])
@pytest.mark.parametrize("directed", [False, True])
def test_thm8_first_sweep_is_gauss_seidel(omega, directed):
    """Thm. 8: the first n pops (queue seeded with every node in index order)
    reproduce one natural-order Gauss-Seidel / SOR sweep from zero on
    (I+L) zhat' = s'."""
    g = synth.chung_lu(300, 1500, 2.3, 71, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "uniform", 72)
    c = 1e-5
    p = oracle.push(g, s, 1e-6, omega=omega, max_pops=g.n, **EPS_SIGMA_C)
    d = oracle.degrees(g)
    z = np.zeros(g.n)
    for i in range(g.n):  # Eq. (gauss) with the SOR blend
        lo, hi = g.row_ptr[i], g.row_ptr[i + 1]
        w = np.ones(hi - lo) if g.w is None else g.w[lo:hi].astype(np.float64)
        gs_val = (s[i] + c + np.dot(w, z[g.col[lo:hi]])) / (1 + d[i])
        z[i] = (1 - omega) * z[i] + omega * gs_val
    assert np.max(np.abs((p["z"] + c) - z)) <= 1e-14


@pytest.mark.parametrize("directed", [False, True])
def test_lemma6_one_sided_bound_bli(directed):
    """omega = 1 keeps r >= 0, so (1 - eps') z' <= zhat' <= z' (Lemma 6)."""
    g = synth.chung_lu(1500, 7000, 2.3, 81, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "uniform", 82)
    eps, c = 1e-3, 1e-5
    epsp = 1e-5 * eps / (c + 1e-5)
    zt = oracle.exact(g, s) + c
    p = oracle.push(g, s, eps, omega=1.0, **EPS_SIGMA_C)
    zh = p["z"] + c
    assert np.all(p["r"] >= 0)
    assert np.all(zh <= zt + 1e-14)
    assert np.all(zh >= (1 - epsp) * zt - 1e-14)


@pytest.mark.parametrize("omega,directed", [(1.2, False), (1.5, False), (1.9, False),
                                            (1.2, True), (0.8, True)])
def test_lemma7_two_sided_bound_sor(omega, directed):
    """|zhat' - z'| <= eps' z' at termination (Lemma 7), and the returned z has
    relative error <= eps wherever z >= sigma (the ImprovedBLI lemma)."""
    g = synth.chung_lu(1500, 7000, 2.3, 91, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "pareto", 92)
    eps, c = 1e-3, 1e-5
    epsp = 1e-5 * eps / (c + 1e-5)
    zt = oracle.exact(g, s)
    p = oracle.push(g, s, eps, omega=omega, max_edge_visits=10**8, **EPS_SIGMA_C)
    assert not p["capped"] and not p["diverged"]
    assert np.all(np.abs(p["r"]) <= epsp * (s + c))
    assert np.all(np.abs(p["z"] - zt) <= epsp * (zt + c) + 1e-14)
    assert oracle.max_rel_error(p["z"], zt, floor=1e-5) <= eps


def test_brute_force_all_graphs_on_four_nodes():
    """Every undirected graph on 4 labelled nodes: push, CG and Gauss-Seidel
    against the dense definition."""
    pairs = list(itertools.combinations(range(4), 2))
    s = np.array([0.1, 0.0, 0.8, 0.45])
    for mask in range(1 << len(pairs)):
        arcs = [pairs[b] for b in range(len(pairs)) if mask >> b & 1]
        g = graphs.from_arcs(4, arcs)
        zd = oracle.dense_solve(g, s)
        for omega in (1.0, 1.5):
            p = oracle.push(g, s, 1e-9, omega=omega, **EPS_SIGMA_C)
            assert np.all(np.abs(p["z"] - zd) <= 0.5e-9 * (zd + 1e-5) + 1e-15)
        assert np.allclose(oracle.gs(g, s)[0], zd, atol=1e-12)
        assert np.allclose(oracle.cg(g, s)[0], zd, atol=1e-12)


def test_zero_opinions_terminate_with_shift():
    """The shift c keeps every threshold positive, so a node with s_v = 0 still
    terminates (Sec. 5.1.3); the estimate is exact to eps' (z' + c)."""
    g = synth.barabasi_albert(200, 2, 5)
    s = np.zeros(g.n)
    s[::7] = 1.0
    p = oracle.push(g, s, 1e-4, max_edge_visits=10**8, **EPS_SIGMA_C)
    assert not p["capped"]
    zt = oracle.exact(g, s)
    assert np.all(np.abs(p["z"] - zt) <= 0.5e-4 * (zt + 1e-5) + 1e-15)


def test_directed_over_relaxation_divergence_is_reported():
    """SOR convergence is only argued for symmetric I+L (Sec. 5.2); on this
    directed graph omega = 1.5 diverges and the oracle must say so rather than
    return the NaNs that drained its queue."""
    g = synth.chung_lu(1500, 7000, 2.3, 91, directed=True, weighted=True)
    s = synth.opinions(g.n, "pareto", 92)
    p = oracle.push(g, s, 1e-3, omega=1.5, max_edge_visits=10**8, **EPS_SIGMA_C)
    assert p["capped"] or p["diverged"]


def test_push_cap_reports_not_converged():
    g = synth.barabasi_albert(500, 3, 6)
    s = synth.opinions(g.n, "uniform", 6)
    p = oracle.push(g, s, 1e-8, max_pops=100)
    assert p["capped"] and p["pops"] == 100


def test_warm_start_from_exact_solution_needs_no_pushes():
    g = synth.chung_lu(2000, 9000, 2.3, 12)
    s = synth.opinions(g.n, "uniform", 13)
    zt = oracle.exact(g, s)
    p = oracle.push(g, s, 1e-6, z0=zt, **EPS_SIGMA_C)
    assert p["pops"] == 0
    p2 = oracle.push(g, s, 1e-6, z0=s, **EPS_SIGMA_C)
    assert oracle.max_rel_error(p2["z"], zt) <= 1e-6


# ------------------------------------------------------------------ metrics
def _metrics_by_definition(g, s, z):
    """Table 1 written out with Python loops over an explicit edge set."""
    n = g.n
    mean = sum(z) / n
    P = sum((zi - mean) ** 2 for zi in z)
    I = sum((z[i] - s[i]) ** 2 for i in range(n))
    C = sum(zi * zi for zi in z)
    edges = {}
    for i in range(n):
        for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = int(g.col[k])
            a = 1.0 if g.w is None else float(g.w[k])
            key = (i, j) if g.directed else (min(i, j), max(i, j))
            edges[key] = a
    D = sum(a * (z[i] - z[j]) ** 2 for (i, j), a in edges.items())
    return dict(P=P, D=D, I=I, C=C)


@pytest.mark.parametrize("directed,weighted", [(False, False), (True, True), (False, True)])
def test_metrics_match_definition(directed, weighted):
    g = graphs.random_graph(40, 0.2, 101, directed=directed, weighted=weighted)
    s = synth.opinions(g.n, "uniform", 102)
    z = oracle.dense_solve(g, s)
    got = oracle.metrics(g, s, z)
    want = _metrics_by_definition(g, s, z)
    for k in "PDIC":
        assert abs(got[k] - want[k]) <= 1e-12 * max(1.0, abs(want[k]))


@pytest.mark.parametrize("n", [3, 8, 25])
def test_metrics_complete_graph_closed_form(n):
    g = graphs.complete(n)
    s = synth.opinions(n, "beta", 3, a=2, b=2)
    z = oracle.dense_solve(g, s)
    m = oracle.metrics(g, s, z)
    S = s.sum()
    assert np.isclose(m["P"], ((s - s.mean()) ** 2).sum() / (n + 1) ** 2, rtol=1e-12)
    D = sum((s[i] - s[j]) ** 2 for i in range(n) for j in range(i + 1, n)) / (n + 1) ** 2
    assert np.isclose(m["D"], D, rtol=1e-12)
    assert np.isclose(m["I"], ((S - n * s) ** 2).sum() / (n + 1) ** 2, rtol=1e-12)


def test_metrics_conservation_undirected():
    """s = (I+L) z gives s^T s = C + 2D + I for a symmetric Laplacian, and
    P = C - n mean^2."""
    g = synth.chung_lu(3000, 15000, 2.3, 111, weighted=True)
    s = synth.opinions(g.n, "bimodal", 112)
    z = oracle.exact(g, s)
    m = oracle.metrics(g, s, z)
    assert abs(m["C"] + 2 * m["D"] + m["I"] - s @ s) <= 1e-9 * (s @ s)
    assert abs(m["P"] - (m["C"] - g.n * m["mean"] ** 2)) <= 1e-10 * m["C"]


def test_certificate_bounds_relative_error():
    """certificate() <= 1 certifies the relative error of Lemma 7 / ImprovedBLI."""
    g = synth.chung_lu(3000, 15000, 2.3, 121, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 122)
    zt = oracle.exact(g, s)
    assert oracle.certificate(g, s, zt, 1e-6) < 1e-3
    for omega in (1.0, 1.4):
        p = oracle.push(g, s, 1e-4, omega=omega, **EPS_SIGMA_C)
        cert = oracle.certificate(g, s, p["z"], 1e-4)
        assert cert <= 1.0 + 1e-6
        assert oracle.max_rel_error(p["z"], zt) <= 1e-4
    # a perturbed z fails it
    bad = zt * (1 + 3e-4)
    assert oracle.certificate(g, s, bad, 1e-4) > 1.0


@pytest.mark.parametrize("c,sigma", [(1e-5, 1e-5), (3e-5, 1e-5), (0.0, 1e-5), (1e-5, 4e-5)])
def test_certificate_value_with_a_planted_residual(c, sigma):
    """Plant the residual: z = z* - (I+L)^{-1} r gives s - (I+L) z = r
    (Lemma 1).  With r_v = t eps (s_v + c) for a constant t, the ratio of
    Alg. 3's threshold test after Alg. 2's shift is |r_v| / (eps' (s_v + c)) =
    t (c + sigma) / sigma at every node, eps' = sigma eps / (c + sigma).  Using
    eps for eps', s for s + c, or a residual of the unshifted estimate gives
    another number."""
    g = synth.chung_lu(600, 3000, 2.3, 123, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 124)
    s[::5] = 0.0  # nodes where s and s + c differ by a factor
    if c == 0.0:
        s = s + 0.05
    eps, t = 1e-3, 0.75
    r = t * eps * (s + c) * np.where(np.arange(g.n) % 2 == 0, 1.0, -1.0)
    z = oracle.dense_solve(g, s) - oracle.dense_solve(g, r)
    want = t * (c + sigma) / sigma
    assert abs(oracle.certificate(g, s, z, eps, sigma=sigma, c=c) - want) <= 1e-6 * want


def test_fj_iterate_is_equation_one():
    """One synchronous step of Eq. (1) by hand on a weighted directed path, and
    many steps converge to the equilibrium of Lemma 1."""
    g = graphs.chain(4, 0.5)
    s = np.array([0.2, 0.4, 0.6, 0.8])
    z = np.array([1.0, 0.0, 1.0, 0.0])
    want = np.array([(0.2 + 0.5 * 0.0) / 1.5, (0.4 + 0.5 * 1.0) / 1.5, (0.6 + 0.5 * 0.0) / 1.5, 0.8])
    assert np.allclose(oracle.fj_iterate(g, s, z, 1), want, atol=1e-15)
    g2 = synth.chung_lu(2000, 9000, 2.3, 131, directed=True, weighted=True)
    s2 = synth.opinions(g2.n, "uniform", 132)
    assert np.max(np.abs(oracle.fj_iterate(g2, s2, s2, 400) - oracle.exact(g2, s2))) <= 1e-9


# ----------------------------------------------------------------- stress
def test_stress_hand_example():
    """Path 0-1-2 with unit weights, z = (0.1, 0.4, 0.9), s = (0, 0.5, 1):
    stress = (0.01 + 0.09, 0.01 + 0.09 + 0.25, 0.01 + 0.25), worked by hand."""
    g = synth.CSRGraph(3, np.array([0, 1, 3, 4], np.int32), np.array([1, 0, 2, 1], np.int32), None, False)
    st = oracle.stress(g, [0.0, 0.5, 1.0], [0.1, 0.4, 0.9])
    assert np.allclose(st, [0.10, 0.35, 0.26], rtol=0, atol=1e-15)


@pytest.mark.parametrize("directed", [False, True])
def test_stress_total_against_measures(directed):
    """Sum of the per-node stress equals I + 2D on an undirected graph (each
    edge sits in two rows) and I + D on a directed one, with D per Table 1
    as the C measures compute it."""
    g = synth.chung_lu(3000, 15000, 2.2, 81 + directed, directed=directed, weighted=True)
    s = synth.opinions(g.n, "uniform", 82)
    z = oracle.exact(g, s)
    m = oracle.metrics(g, s, z)
    total = oracle.stress(g, s, z).sum()
    want = m["I"] + (m["D"] if directed else 2.0 * m["D"])
    assert abs(total - want) <= 1e-12 * want


def test_equilibrium_minimises_each_node_stress():
    """At the equilibrium every node's opinion minimises its own stress with
    the others held fixed (the FJ update of Eq. (1) is that minimiser), so
    moving one node's z either way raises its stress."""
    g = synth.chung_lu(500, 2500, 2.3, 83, weighted=True)
    s = synth.opinions(g.n, "beta", 84, a=2, b=2)
    z = oracle.exact(g, s)
    base = oracle.stress(g, s, z)
    for i in (0, 7, 123, 499):
        for delta in (1e-3, -1e-3):
            zp = z.copy()
            zp[i] += delta
            assert oracle.stress(g, s, zp)[i] > base[i]


# ------------------------------------------------ spectral radius and omega
@pytest.mark.parametrize("k", [3, 8, 32])
def test_spectral_radius_even_cycle(k):
    """Unit-weight cycle: (I+D)^{-1} A = A / 3, whose largest eigenvalue is 2/3."""
    assert abs(oracle.jacobi_spectral_radius(graphs.cycle(2 * k)) - 2.0 / 3.0) <= 1e-12


@pytest.mark.parametrize("n", [2, 5, 40])
def test_spectral_radius_complete_graph(n):
    """K_n: (I+D)^{-1} A = A / n with eigenvalues (n-1)/n and -1/n."""
    assert abs(oracle.jacobi_spectral_radius(graphs.complete(n)) - (n - 1) / n) <= 1e-12


@pytest.mark.parametrize("k", [1, 10, 500])
def test_spectral_radius_star(k):
    """Star with k leaves: lambda x_c = k x_l / (1+k) and lambda x_l = x_c / 2,
    so mu^2 = k / (2 (k+1))."""
    assert abs(oracle.jacobi_spectral_radius(graphs.star(k)) - np.sqrt(k / (2.0 * (k + 1)))) <= 1e-12


def test_spectral_radius_sparse_path_closed_forms():
    """n > 2000 takes the sparse (Lanczos / Arnoldi) path; pin it to closed
    forms: the even cycle C_4000 (mu = 2/3), K_2100 (mu = 2099/2100) and the
    star with 3000 leaves (mu^2 = k / (2 (k+1)))."""
    assert abs(oracle.jacobi_spectral_radius(graphs.cycle(4000)) - 2.0 / 3.0) <= 1e-12
    assert abs(oracle.jacobi_spectral_radius(graphs.complete(2100)) - 2099.0 / 2100.0) <= 1e-12
    k = 3000
    assert abs(oracle.jacobi_spectral_radius(graphs.star(k)) - np.sqrt(k / (2.0 * (k + 1)))) <= 1e-12


def test_spectral_radius_sparse_path_directed_secular_equation():
    """Directed complete graph on n = 2100 nodes where node i listens to every
    other node with its own weight w_i: (I+D)^{-1} A = diag(al) (1 1^T - I) with
    al_i = w_i / (1 + (n-1) w_i).  lambda is an eigenvalue iff 1 1^T - diag(1 +
    lambda / al) is singular, i.e. sum_i al_i / (al_i + lambda) = 1; the left
    side falls from n to 0 on lambda > 0, so the Perron root is its one
    positive root, found here by bisection."""
    n = 2100
    rng = np.random.default_rng(5)
    wr = rng.uniform(0.5, 1.5, n).astype(np.float32)
    arcs = [(i, j) for i in range(n) for j in range(n) if i != j]
    g = graphs.from_arcs(n, arcs, [wr[i] for i, _ in arcs], directed=True)
    wf = wr.astype(np.float64)
    al = wf / (1.0 + (n - 1) * wf)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(al / (al + mid)) > 1.0:
            lo = mid
        else:
            hi = mid
    assert abs(oracle.jacobi_spectral_radius(g) - lo) <= 1e-12


def test_spectral_radius_sparse_path_inside_row_sum_bound():
    g = synth.chung_lu(2500, 12000, 2.2, 85, directed=True, weighted=True)
    mu = oracle.jacobi_spectral_radius(g)
    d = oracle.degrees(g)
    assert 0.0 < mu <= np.max(d / (1.0 + d)) + 1e-12


@pytest.mark.parametrize("mu", [0.0, 0.3, 2.0 / 3.0, 0.9, 0.99])
def test_optimal_omega_equals_young_form(mu):
    """Eq. (optimal-omega) equals 2 / (1 + sqrt(1 - mu^2)): with q = mu/(1+t),
    t = sqrt(1-mu^2), 1 + q^2 = (1 + 2t + t^2 + mu^2)/(1+t)^2 = 2/(1+t)."""
    assert abs(oracle.optimal_omega(mu) - 2.0 / (1.0 + np.sqrt(1.0 - mu * mu))) <= 1e-14
    assert 1.0 <= oracle.optimal_omega(mu) < 2.0


# ------------------------------------------------- a-posteriori metric bounds
def _measures_dense(g, s, z):
    return dict(**_metrics_by_definition(g, s, z), mean=float(np.mean(z)))


def _box(g, s, zh, c):
    """Residual level and per-node radius from the dense matrix (Lemma 7)."""
    r = s - oracle.dense_matrix(g) @ zh
    tau = float(np.max(np.abs(r) / (s + c)))
    return tau, tau * (zh + c) / (1.0 - tau)


@pytest.mark.parametrize("directed,weighted", [(False, False), (True, True), (False, True)])
def test_bounds_contain_exact_measures(directed, weighted):
    """The measures of the exact z lie within the bounds around a perturbed z,
    and the exact z within the per-node radius of Lemma 7."""
    c = 1e-5
    g = graphs.random_graph(30, 0.2, 131, directed=directed, weighted=weighted)
    s = synth.opinions(g.n, "uniform", 132)
    zt = oracle.dense_solve(g, s)
    rng = np.random.default_rng(133)
    for rel in (1e-6, 1e-4, 1e-3):
        zh = zt * (1.0 + rel * rng.uniform(-1, 1, g.n))
        bound, tau = oracle.metrics_bounds(g, s, zh, c)
        t2, b = _box(g, s, zh, c)
        assert tau < 1.0 and np.isclose(tau, t2, rtol=1e-9)
        assert np.all(np.abs(zh - zt) <= b * (1 + 1e-12))
        mh, mt = _measures_dense(g, s, zh), _measures_dense(g, s, zt)
        for k in ("P", "D", "I", "C", "mean"):
            assert abs(mh[k] - mt[k]) <= bound[k] * (1 + 1e-12) + 1e-15, (rel, k)


@pytest.mark.parametrize("directed,seed", [(False, 141), (True, 142), (False, 143)])
def test_bounds_against_brute_force_over_box_vertices(directed, seed):
    """Over all 2^n moves e_v = +-b_v: the C, I and mean bounds equal the
    largest change, the P and D bounds are at least as large (the convex
    measures take their largest increase at a vertex of the box)."""
    c = 1e-5
    g = graphs.random_graph(7, 0.5, seed, directed=directed, weighted=True)
    s = synth.opinions(g.n, "uniform", seed + 1)
    zt = oracle.dense_solve(g, s)
    zh = zt * (1.0 + 1e-3 * np.random.default_rng(seed + 2).uniform(-1, 1, g.n))
    bound, tau = oracle.metrics_bounds(g, s, zh, c)
    assert tau < 1.0
    _, b = _box(g, s, zh, c)
    base = _measures_dense(g, s, zh)
    worst = dict.fromkeys(base, 0.0)
    for signs in itertools.product((-1.0, 1.0), repeat=g.n):
        m = _measures_dense(g, s, zh + np.array(signs) * b)
        for k in worst:
            worst[k] = max(worst[k], abs(m[k] - base[k]))
    for k in ("C", "I", "mean"):
        assert np.isclose(bound[k], worst[k], rtol=1e-9), k
    for k in ("P", "D"):
        assert bound[k] >= worst[k] * (1 - 1e-12), k


@pytest.mark.parametrize("n", [2, 6])
def test_polarization_bound_attained_at_a_constant_estimate(n):
    """With every z_v equal the first-order change of P vanishes and moves of
    alternating sign keep the mean: the P bound is the largest change."""
    c = 1e-5
    g = graphs.cycle(n) if n > 2 else graphs.from_arcs(2, [(0, 1)])
    s = np.full(n, 0.4)  # z_exact = s (L 1 = 0)
    zh = np.full(n, 0.4 * (1.0 + 1e-3))
    bound, tau = oracle.metrics_bounds(g, s, zh, c)
    assert tau < 1.0
    _, b = _box(g, s, zh, c)
    base = _measures_dense(g, s, zh)["P"]
    worst = max(abs(_measures_dense(g, s, zh + np.array(sg) * b)["P"] - base)
                for sg in itertools.product((-1.0, 1.0), repeat=n))
    assert np.isclose(bound["P"], worst, rtol=1e-9)


@pytest.mark.parametrize("w", [1.0, 0.3])
def test_disagreement_bound_attained_on_one_edge(w):
    """On a single edge the two ends can move apart by b_1 + b_2: the D bound
    is the change itself (an undirected edge counted once)."""
    c = 1e-5
    g = graphs.from_arcs(2, [(0, 1)], [w])
    s = np.array([0.9, 0.2])
    zt = oracle.dense_solve(g, s)
    zh = zt + np.array([2e-3, -1e-3])
    bound, _ = oracle.metrics_bounds(g, s, zh, c)
    _, b = _box(g, s, zh, c)
    sgn = np.sign(zh[0] - zh[1])
    moved = _measures_dense(g, s, zh + np.array([sgn * b[0], -sgn * b[1]]))
    assert np.isclose(bound["D"], abs(moved["D"] - _measures_dense(g, s, zh)["D"]), rtol=1e-12)


@pytest.mark.parametrize("directed", [False, True])
def test_bounds_equality_case_of_lemma7(directed):
    """z' = (1 - t) z_exact' leaves the residual t s', so tau = t, the radius
    b_v equals the error z_exact_v - z_v, and the C bound is the change in C."""
    c, t = 1e-5, 2e-3
    g = graphs.random_graph(25, 0.25, 151, directed=directed, weighted=True)
    s = synth.opinions(g.n, "uniform", 152)
    zt = oracle.dense_solve(g, s)
    zh = (1.0 - t) * (zt + c) - c
    bound, tau = oracle.metrics_bounds(g, s, zh, c)
    assert np.isclose(tau, t, rtol=1e-9)
    m0, m1 = _measures_dense(g, s, zh), _measures_dense(g, s, zt)
    assert np.isclose(bound["C"], m1["C"] - m0["C"], rtol=1e-8)
    assert np.isclose(bound["mean"], m1["mean"] - m0["mean"], rtol=1e-8)


def test_bounds_of_a_certified_push():
    """A push certified at eps has tau <= eps' = sigma eps / (c + sigma), and
    the exact measures lie within the bounds around its z."""
    g = synth.chung_lu(2000, 10000, 2.3, 161, weighted=True)
    s = synth.opinions(g.n, "uniform", 162)
    zt = oracle.exact(g, s)
    eps = 1e-3
    p = oracle.push(g, s, eps, omega=1.3, **EPS_SIGMA_C)
    bound, tau = oracle.metrics_bounds(g, s, p["z"], EPS_SIGMA_C["c"])
    epsp = EPS_SIGMA_C["sigma"] * eps / (EPS_SIGMA_C["c"] + EPS_SIGMA_C["sigma"])
    assert tau <= epsp * (1 + 1e-9)
    mh, mt = oracle.metrics(g, s, p["z"]), oracle.metrics(g, s, zt)
    for k in ("P", "D", "I", "C", "mean"):
        assert abs(mh[k] - mt[k]) <= bound[k], k


def test_bounds_infinite_without_a_contraction():
    g = graphs.complete(4)
    s = np.array([0.1, 0.2, 0.3, 0.4])
    bound, tau = oracle.metrics_bounds(g, s, np.full(4, 5.0), 1e-5)
    assert tau >= 1.0 and all(np.isinf(v) for v in bound.values())
