"""FP64 reference of the warm-start network (test infrastructure only).

The paper has no learned component; this network is an extension that only
proposes a starting estimate.  By Lemma 4 any starting estimate is valid and
by Lemma 7 the residual certificate decides the result, so the network never
changes what is computed, only how long the push runs.  This module is the
plain definition the GPU kernels are checked against; its gradients are pinned
by central finite differences and its forward by a loop form
(tests/test_oracle_mpnn.py).  Parity with the paper: unpinned (the paper has
no such network).

Definition (all arrays FP64, n nodes, CSR of A with weights a_ij):
  d_v   = sum_j a_vj
  nbr_v(x) = sum_j a_vj x_j / d_v   (0 when d_v = 0)
  ns    = nbr(s)
  z1_v  = (s_v + d_v ns_v) / (1 + d_v)      one step of Eq. (1) from s
  X0_v  = [s_v, ns_v, z1_v, log1p d_v, 1/(1+d_v), mean(s), 1, 0]      (n x 8)
  H1 = relu(X0 W1 + b1)                      (n x 64)   layer 1
  P  = H1 Wp                                 (n x 16)   message of layer 2
  M  = nbr(P)                                (n x 16)
  H2 = relu([H1 | M] W2 + b2)                (n x 64)   layer 2
  o  = H2 u + c0
  z0 = min(s) + (max(s) - min(s)) sigmoid(o)   (inside [min s, max s], where
       the equilibrium lies: (I+L)^{-1} is row-stochastic, Sec. 3.3)
  loss = mean_v w_v (z0_v - z_v)^2,  w_v = 1 (rel_floor <= 0) or
         1 / (z_v + rel_floor)^2 (relative error with a floor; the
         certificate is relative, so nodes with a small z weigh more)
Layer 1's message is the opinion itself (ns), layer 2's a learned 16-wide
projection of the hidden state.  Parameters are one flat FP32/FP64 vector:
W1 (8x64 row-major), b1 (64), Wp (64x16), W2 (80x64), b2 (64), u (64), c0 (1).
"""
import numpy as np

F_IN, HID, MSG = 8, 64, 16
SIZES = [("W1", (F_IN, HID)), ("b1", (HID,)), ("Wp", (HID, MSG)), ("W2", (HID + MSG, HID)), ("b2", (HID,)),
         ("u", (HID,)), ("c0", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def offsets():
    """name -> (first, one past last) in the flat parameter vector."""
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = (off, off + k)
        off += k
    return out


def unpack(p):
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[off:off + k], dtype=np.float64).reshape(shape)
        off += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    d = {"W1": rng.normal(0, np.sqrt(2.0 / F_IN), (F_IN, HID)), "b1": np.zeros(HID),
         "Wp": rng.normal(0, np.sqrt(1.0 / HID), (HID, MSG)),
         "W2": rng.normal(0, np.sqrt(2.0 / (HID + MSG)), (HID + MSG, HID)), "b2": np.zeros(HID),
         "u": rng.normal(0, np.sqrt(1.0 / HID), HID), "c0": np.zeros(1)}
    return pack(d)


def _adjacency(g):
    import scipy.sparse as sp
    w = np.ones(g.nnz) if g.w is None else g.w.astype(np.float64)
    return sp.csr_matrix((w, g.col, g.row_ptr), shape=(g.n, g.n))


def neighbour_mean_matrix(g):
    """Sparse operator N with (N x)_v = sum_j a_vj x_j / d_v (0 if d_v = 0), and d."""
    import scipy.sparse as sp
    A = _adjacency(g)
    d = np.asarray(A.sum(axis=1)).ravel()
    inv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    return sp.diags(inv) @ A, d


def features(g, s):
    N, d = neighbour_mean_matrix(g)
    s = np.asarray(s, dtype=np.float64)
    ns = N @ s
    X = np.zeros((g.n, F_IN))
    X[:, 0] = s
    X[:, 1] = ns
    X[:, 2] = (s + d * ns) / (1.0 + d)
    X[:, 3] = np.log1p(d)
    X[:, 4] = 1.0 / (1.0 + d)
    X[:, 5] = s.mean()
    X[:, 6] = 1.0
    return X


def forward(g, s, p):
    prm = unpack(p)
    N, _ = neighbour_mean_matrix(g)
    X0 = features(g, s)
    Y1 = X0 @ prm["W1"] + prm["b1"]
    H1 = np.maximum(Y1, 0.0)
    P = H1 @ prm["Wp"]
    M = N @ P
    A2 = np.hstack([H1, M])
    Y2 = A2 @ prm["W2"] + prm["b2"]
    H2 = np.maximum(Y2, 0.0)
    o = H2 @ prm["u"] + prm["c0"][0]
    lo, hi = float(np.min(s)), float(np.max(s))
    sg = 1.0 / (1.0 + np.exp(-o))
    z0 = lo + (hi - lo) * sg
    return dict(N=N, X0=X0, Y1=Y1, H1=H1, P=P, M=M, A2=A2, Y2=Y2, H2=H2, o=o, sg=sg, z0=z0, lo=lo, hi=hi)


def loss_weights(z_target, rel_floor=0.0):
    z = np.asarray(z_target, dtype=np.float64)
    return np.ones_like(z) if rel_floor <= 0.0 else 1.0 / (z + rel_floor) ** 2


def loss_and_grad(g, s, p, z_target, rel_floor=0.0):
    """The (weighted) mean squared error of z0 against z_target and its
    gradient (flat), by the chain rule through the definition above."""
    prm = unpack(p)
    f = forward(g, s, p)
    n = g.n
    r = f["z0"] - np.asarray(z_target, dtype=np.float64)
    wv = loss_weights(z_target, rel_floor)
    loss = float(np.mean(wv * r * r))
    dz0 = 2.0 * wv * r / n
    do = dz0 * (f["hi"] - f["lo"]) * f["sg"] * (1.0 - f["sg"])
    grads = {"u": f["H2"].T @ do, "c0": np.array([do.sum()])}
    dY2 = np.outer(do, prm["u"]) * (f["Y2"] > 0)
    grads["W2"] = f["A2"].T @ dY2
    grads["b2"] = dY2.sum(axis=0)
    dA2 = dY2 @ prm["W2"].T
    dM = dA2[:, HID:]
    dP = f["N"].T @ dM
    grads["Wp"] = f["H1"].T @ dP
    dH1 = dA2[:, :HID] + dP @ prm["Wp"].T
    dY1 = dH1 * (f["Y1"] > 0)
    grads["W1"] = f["X0"].T @ dY1
    grads["b1"] = dY1.sum(axis=0)
    return loss, pack(grads)
