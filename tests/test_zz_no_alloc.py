"""fj_metrics_noalloc (no workspace, static device scratch) against fj_metrics.

Both run the same kernels and fixed-order reductions, so the measures must be
bitwise equal; they are also held to the oracle's measures of the same z.  Two
calls in a row, the second on a smaller graph, check that the shared static
array needs no clearing between calls; a graph whose partial sums exceed the
array is rejected with a clear error.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(n, m_edges, seed, directed):
    g = synth.chung_lu(n, m_edges, 2.3 if not directed else 2.1, seed, directed=directed, weighted=directed)
    s = synth.opinions(g.n, "bimodal", seed)
    z = np.clip(s + 0.05 * synth.opinions(g.n, "uniform", seed + 1) - 0.025, 0.0, 1.0)
    return g, s, z


def test_noalloc_matches_workspace_entry_twice_second_smaller():
    import paper_2507_14864_amd as fj
    for n, m, seed, directed in ((300_000, 3_000_000, 71, False), (40_000, 300_000, 72, True)):
        g, s, z = _case(n, m, seed, directed)
        G = fj.Graph.from_host(g, DEV)
        need, cap = fj.metrics_noalloc_bytes(G)
        print(f"noalloc case n={g.n} nnz={g.nnz} directed={directed} need={need} cap={cap}", flush=True)
        assert 0 < need <= cap
        sd = torch.from_numpy(s).to(DEV)
        zd = torch.from_numpy(z).to(DEV)
        ref = fj.metrics(G, sd, zd)
        got = fj.metrics_noalloc(G, sd, zd)
        for k in ("P", "D", "I", "C", "mean"):
            assert got[k] == ref[k], (k, got[k], ref[k])
        mo = oracle.metrics(g, s, z)
        for k in "PDIC":
            assert abs(got[k] - mo[k]) <= 1e-12 * abs(mo[k]), (k, got[k], mo[k])
        torch.cuda.synchronize()


def test_noalloc_empty_graph_and_rejection():
    import paper_2507_14864_amd as fj
    # no nodes: zeros, no launch
    G0 = fj.Graph(torch.zeros(1, dtype=torch.int32, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV))
    e = torch.zeros(0, dtype=torch.float64, device=DEV)
    assert fj.metrics_noalloc(G0, e, e) == {"P": 0.0, "D": 0.0, "I": 0.0, "C": 0.0, "mean": 0.0}
    # an edgeless graph large enough that its partial sums exceed the array
    n = 80_000_000
    G = fj.Graph(torch.zeros(n + 1, dtype=torch.int32, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV))
    need, cap = fj.metrics_noalloc_bytes(G)
    print(f"noalloc rejection n={n} need={need} cap={cap}", flush=True)
    assert need > cap
    s = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(fj.FJError) as ei:
        fj.metrics_noalloc(G, s, s)
    assert ei.value.status == 2 and "static scratch" in str(ei.value)
