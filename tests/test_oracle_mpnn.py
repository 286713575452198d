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
    prm = mpnn.unpack(p)
    n = g.n
    w = lambda k: 1.0 if g.w is None else float(g.w[k])
    d = np.zeros(n)
    din = np.zeros(n)
    for i in range(n):
        for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
            d[i] += w(k)
            din[g.col[k]] += w(k)

    def nbr(x):
        out = np.zeros_like(x)
        for i in range(n):
            for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
                out[i] += w(k) * x[g.col[k]]
            if d[i] > 0:
                out[i] /= d[i]
        return out

    X = np.zeros((n, 8))
    for i in range(n):
        X[i] = [s[i], 0, np.log1p(d[i]), np.log1p(din[i]), 1 / (1 + d[i]), np.mean(s), 1, 0]
    X[:, 1] = nbr(np.asarray(s, float))
    H1 = np.maximum(np.hstack([X, nbr(X)]) @ prm["W1"] + prm["b1"], 0)
    H2 = np.maximum(np.hstack([H1, nbr(H1)]) @ prm["W2"] + prm["b2"], 0)
    o = H2 @ prm["u"] + prm["c0"][0]
    return min(s) + (max(s) - min(s)) / (1 + np.exp(-o))


def test_forward_matches_loop_definition():
    g = graphs.random_graph(25, 0.2, 3, directed=True, weighted=True)
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
    loss, grad = mpnn.loss_and_grad(g, s, p, zt)
    rng = np.random.default_rng(12)
    idx = np.concatenate([rng.choice(mpnn.N_PARAMS, 60, replace=False), [mpnn.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mpnn.loss_and_grad(g, s, p + e, zt)
        lm, _ = mpnn.loss_and_grad(g, s, p - e, zt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, grad[i])
