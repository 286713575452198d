"""Pins for the FP64 warm-start network reference (oracle/mpnn.py).

The network is not in the paper (parity unpinned there); its reference is
pinned by (a) an independent forward written with explicit Python loops over
the edge list and (b) central finite differences of the loss for the gradient.
"""
import numpy as np

import synth
from oracle import mpnn
from tests import graphs


def _loop_forward(g, s, p):
    """The network written out with explicit loops over rows, arcs and units."""
    prm = mpnn.unpack(p)
    n = g.n
    w = lambda k: 1.0 if g.w is None else float(g.w[k])
    d = np.zeros(n)
    for i in range(n):
        for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
            d[i] += w(k)

    def nbr(x):
        out = np.zeros_like(x)
        for i in range(n):
            for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
                out[i] += w(k) * x[g.col[k]]
            if d[i] > 0:
                out[i] /= d[i]
        return out

    ns = nbr(np.asarray(s, float))
    mean = sum(s) / n
    X = np.zeros((n, 8))
    for i in range(n):
        X[i] = [s[i], ns[i], (s[i] + d[i] * ns[i]) / (1 + d[i]), np.log1p(d[i]), 1 / (1 + d[i]), mean, 1, 0]
    H1 = np.zeros((n, 64))
    for i in range(n):
        for c in range(64):
            H1[i, c] = max(0.0, sum(X[i, f] * prm["W1"][f, c] for f in range(8)) + prm["b1"][c])
    P = np.zeros((n, 16))
    for i in range(n):
        for j in range(16):
            P[i, j] = sum(H1[i, c] * prm["Wp"][c, j] for c in range(64))
    M = nbr(P)
    z0 = np.zeros(n)
    for i in range(n):
        o = prm["c0"][0]
        for c in range(64):
            y = prm["b2"][c] + sum(H1[i, m] * prm["W2"][m, c] for m in range(64)) + \
                sum(M[i, j] * prm["W2"][64 + j, c] for j in range(16))
            o += max(0.0, y) * prm["u"][c]
        z0[i] = min(s) + (max(s) - min(s)) / (1 + np.exp(-o))
    return z0


def test_forward_matches_loop_definition():
    g = graphs.random_graph(12, 0.3, 3, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 4)
    p = mpnn.init_params(5)
    assert np.allclose(mpnn.forward(g, s, p)["z0"], _loop_forward(g, s, p), atol=1e-12)


def test_output_stays_inside_opinion_range():
    g = synth.chung_lu(500, 3000, 2.1, 6, directed=True, weighted=True)
    s = synth.opinions(g.n, "bimodal", 7)
    for seed in range(3):
        z0 = mpnn.forward(g, s, mpnn.init_params(seed) * 3.0)["z0"]
        assert z0.min() >= s.min() - 1e-15 and z0.max() <= s.max() + 1e-15


def test_gradient_matches_finite_differences():
    g = graphs.random_graph(30, 0.15, 8, directed=True, weighted=True)
    s = synth.opinions(g.n, "uniform", 9)
    zt = synth.opinions(g.n, "uniform", 10)
    p = mpnn.init_params(11)
    p[mpnn.N_PARAMS - 1] = 0.3  # c0 away from a symmetric point
    check_fd(g, s, p, zt, 0.0)
    check_fd(g, s, p, zt, 0.05)


def check_fd(g, s, p, zt, rel_floor):
    loss, grad = mpnn.loss_and_grad(g, s, p, zt, rel_floor)
    rng = np.random.default_rng(12)
    # entries of every block, c0 included
    idx = np.concatenate([rng.integers(a, b, 12) for a, b in mpnn.offsets().values()] + [[mpnn.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mpnn.loss_and_grad(g, s, p + e, zt, rel_floor)
        lm, _ = mpnn.loss_and_grad(g, s, p - e, zt, rel_floor)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, grad[i])


def test_relative_weights_are_the_definition():
    """The weighted loss equals the mean of ((z0 - z)/(z + floor))^2 written out."""
    g = graphs.random_graph(20, 0.2, 13, directed=True, weighted=True)
    s = synth.opinions(g.n, "bimodal", 14)
    zt = synth.opinions(g.n, "uniform", 15)
    p = mpnn.init_params(16)
    z0 = mpnn.forward(g, s, p)["z0"]
    want = sum(((a - b) / (b + 0.01)) ** 2 for a, b in zip(z0, zt)) / g.n
    assert abs(mpnn.loss_and_grad(g, s, p, zt, 0.01)[0] - want) <= 1e-12 * want
