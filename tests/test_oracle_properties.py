"""Property tests of the oracle over random small graphs (Hypothesis).

Every example draws a graph on 1..12 nodes (directed or undirected, unit or
U[0.5, 1.5] weights, any density), opinions with zeros among them, a
relaxation factor in (0, 2) and a target eps, and checks what the paper fixes
for every such input against the dense definition z = (I+L)^{-1} s (Lemma 1):

  * Lemma 4: the tracked residual equals s' - (I+L) zhat' after any number of
    pops, for any omega;
  * Lemma 6: at omega = 1 from zero the residual stays >= 0 and the result
    satisfies (1 - eps') z' <= zhat' <= z';
  * Lemma 7: at termination |zhat' - z'| <= eps' z' for any omega;
  * Thm. 8: the first n pops equal one natural-order SOR sweep from zero;
  * the exact solvers (Gauss-Seidel, and PCG when undirected) against LU;
  * the measures: P = C - n m^2, and s^T s = C + 2D + I when undirected.

Examples are derandomized, so a run is reproducible.
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from tests import graphs  # noqa: E402

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True, print_blob=True)
C = SIGMA = 1e-5


@st.composite
def problems(draw, max_n=12):
    n = draw(st.integers(1, max_n))
    directed = draw(st.booleans())
    weighted = draw(st.booleans())
    p = draw(st.floats(0.0, 1.0))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    arcs, ws = [], []
    for i in range(n):
        for j in range(n):
            if i == j or (not directed and j <= i):
                continue
            if rng.random() < p:
                arcs.append((i, j))
                ws.append(rng.uniform(0.5, 1.5))
    g = graphs.from_arcs(n, arcs, ws if weighted else None, directed)
    s = rng.uniform(0.0, 1.0, n)
    s[rng.random(n) < 0.3] = 0.0  # zero opinions: the case the shift c is for
    return g, s


def _shifted(g, s, zhat):
    """s' - (I+L) zhat' with s' = s + c and zhat' = zhat + c."""
    return oracle.residual(g, s + C, zhat + C)


@SETTINGS
@given(problems(), st.floats(0.05, 1.95), st.integers(0, 200))
def test_lemma4_tracked_residual_at_any_stop(prob, omega, pops):
    g, s = prob
    p = oracle.push(g, s, 1e-6, omega=omega, max_pops=pops, sigma=SIGMA, c=C)
    if p["diverged"]:
        return
    scale = max(1.0, np.max(np.abs(p["z"])), np.max(np.abs(p["r"])))
    assert np.max(np.abs(p["r"] - _shifted(g, s, p["z"])), initial=0.0) <= 1e-12 * scale * (1 + g.nnz)


@SETTINGS
@given(problems(), st.sampled_from([1e-2, 1e-4, 1e-7]))
def test_lemma6_one_sided_at_omega_one(prob, eps):
    g, s = prob
    epsp = SIGMA * eps / (C + SIGMA)
    zt = oracle.dense_solve(g, s) + C
    p = oracle.push(g, s, eps, omega=1.0, sigma=SIGMA, c=C)
    assert not p["capped"] and not p["diverged"]
    zh = p["z"] + C
    assert np.all(p["r"] >= 0.0)
    # the LU reference itself is off by rounding, absolutely: where z = 0
    # exactly (s_v = 0 and no path to a positive opinion) it can return
    # -3e-17, below zhat' = c; hence the 1e-15 absolute slack beside the
    # relative one
    assert np.all(zh <= zt * (1 + 1e-13) + 1e-15)
    assert np.all(zh >= (1 - epsp) * zt * (1 - 1e-13) - 1e-15)


@SETTINGS
@given(problems(), st.floats(0.05, 1.95), st.sampled_from([1e-2, 1e-4, 1e-7]))
def test_lemma7_two_sided_at_termination(prob, omega, eps):
    g, s = prob
    epsp = SIGMA * eps / (C + SIGMA)
    p = oracle.push(g, s, eps, omega=omega, max_edge_visits=2_000_000, sigma=SIGMA, c=C)
    if p["capped"] or p["diverged"]:
        # over-relaxation is only argued to converge for symmetric I+L (Sec. 5.2)
        assert g.directed
        return
    zt = oracle.dense_solve(g, s) + C
    assert np.all(np.abs(p["r"]) <= epsp * (s + C))
    assert np.all(np.abs((p["z"] + C) - zt) <= epsp * zt * (1 + 1e-9) + 1e-15)


@SETTINGS
@given(problems(), st.floats(0.05, 1.95))
def test_thm8_first_n_pops_are_one_sor_sweep(prob, omega):
    g, s = prob
    p = oracle.push(g, s, 1e-9, omega=omega, max_pops=g.n, sigma=SIGMA, c=C)
    M = oracle.dense_matrix(g)
    z = np.zeros(g.n)
    for i in range(g.n):  # Eq. (gauss) blended by omega, newest values first
        gs_val = (s[i] + C - (M[i] @ z - M[i, i] * z[i])) / M[i, i]
        z[i] = (1 - omega) * z[i] + omega * gs_val
    assert np.max(np.abs((p["z"] + C) - z), initial=0.0) <= 1e-13


@SETTINGS
@given(problems())
def test_exact_solvers_against_lu(prob):
    g, s = prob
    zd = oracle.dense_solve(g, s)
    assert np.max(np.abs(oracle.gs(g, s, 1e-13)[0] - zd), initial=0.0) <= 1e-12
    if not g.directed:
        assert np.max(np.abs(oracle.cg(g, s, 1e-13)[0] - zd), initial=0.0) <= 1e-12


@SETTINGS
@given(problems())
def test_measures_identities(prob):
    g, s = prob
    z = oracle.dense_solve(g, s)
    m = oracle.metrics(g, s, z)
    assert abs(m["P"] - (m["C"] - g.n * m["mean"] ** 2)) <= 1e-12 * max(1.0, m["C"])
    if not g.directed:
        assert abs(m["C"] + 2 * m["D"] + m["I"] - s @ s) <= 1e-12 * max(1.0, s @ s)
