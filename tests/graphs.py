"""Small hand-built graphs for tests (CSR, same convention as ``synth``)."""
import numpy as np

from synth import CSRGraph


def from_arcs(n, arcs, weights=None, directed=False):
    """CSR from a list of arcs (i, j) meaning a_ij > 0.  Undirected: each pair
    given once, stored both ways."""
    rows = [[] for _ in range(n)]
    for e, (i, j) in enumerate(arcs):
        a = 1.0 if weights is None else float(weights[e])
        rows[i].append((j, a))
        if not directed:
            rows[j].append((i, a))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col, w = [], []
    for i in range(n):
        rows[i].sort()
        row_ptr[i + 1] = row_ptr[i] + len(rows[i])
        col += [j for j, _ in rows[i]]
        w += [a for _, a in rows[i]]
    return CSRGraph(n, row_ptr, np.array(col, dtype=np.int32),
                    None if weights is None else np.array(w, dtype=np.float32), directed)


def complete(n):
    return from_arcs(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(k):
    return from_arcs(k + 1, [(0, i) for i in range(1, k + 1)])


def chain(n, w):
    """Directed chain: node i listens to node i+1 with weight w."""
    return from_arcs(n, [(i, i + 1) for i in range(n - 1)], [w] * (n - 1), directed=True)


def cycle(n):
    return from_arcs(n, [(i, (i + 1) % n) for i in range(n)])


def random_graph(n, p, seed, directed=False, weighted=False):
    rng = np.random.default_rng(seed)
    arcs, ws = [], []
    for i in range(n):
        for j in range(n if directed else i + 1):
            if directed and j == i:
                continue
            if not directed and j >= i:
                continue
            if rng.random() < p:
                arcs.append((i, j))
                ws.append(rng.uniform(0.5, 1.5))
    return from_arcs(n, arcs, ws if weighted else None, directed)
